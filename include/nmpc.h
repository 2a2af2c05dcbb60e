/*
 * nmpc.h - C ABI of the MI355X parametric interior-point NMPC library.
 *
 * The library re-solves a direct-transcribed optimal control problem whose
 * sparsity never changes (Section 3.1, eqs. 4-6).  Each solve runs the
 * Lifted-KKT primal-dual interior-point method of Section 3.2 / Algorithm 2 on
 * the GPU: model evaluation, condensed KKT assembly (eqs. 14, 17), numeric
 * supernodal Cholesky (eqs. 20-21) and forward/back solves (eqs. 22-25).  The
 * symbolic factorization (ordering, elimination tree, supernodes; eqs. 18-19)
 * is computed once by nmpc_analyze and reused by every later iteration and
 * re-solve, as in Algorithms 1-2.
 *
 * Conventions for every entry point:
 *   - pointers marked "host" are ordinary CPU memory owned by the caller; the
 *     library copies what it needs before returning and never keeps them;
 *   - all floating point is IEEE binary64 (double);
 *   - index arrays are int32 unless stated otherwise, 0-based;
 *   - return value: NMPC_OK (0) on success, a negative NMPC_ERR_* code on a hard
 *     error (nothing changed; nmpc_last_error() gives a message), or, from
 *     nmpc_solve only, a positive solver outcome (the last iterate stays
 *     readable);
 *   - a handle may be used by one host thread at a time.
 */
#ifndef NMPC_H
#define NMPC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t nmpc_status;

enum {
    NMPC_OK = 0,
    /* solver outcomes (nmpc_solve), Algorithm 2 termination */
    NMPC_MAX_ITER = 1,          /* iteration limit reached before eq. (28) held */
    NMPC_LINESEARCH_FAIL = 2,   /* backtracking exhausted (eq. 26) */
    NMPC_REG_FAIL = 3,          /* inertia correction exceeded eta_max (eq. 13, 17) */
    NMPC_NONFINITE = 4,         /* NaN/Inf in a model value */
    /* hard errors */
    NMPC_ERR_INVALID_ARG = -1,
    NMPC_ERR_BAD_ORDER = -2,     /* e.g. solve before analyze */
    NMPC_ERR_STRUCT_MISMATCH = -3,
    NMPC_ERR_NO_DEVICE = -4,     /* no HIP device visible */
    NMPC_ERR_HIP = -5,           /* a HIP runtime call failed */
    NMPC_ERR_OOM = -6,
    NMPC_ERR_UNSUPPORTED = -7
};

/* Problem families.  DISTILLATION and HEATED_PLATE are the two workload
 * families (Sections 4.1 and 4.2 in structure); REFLUX_COLUMN is the paper's
 * own distillation case study of Section 4.1 as its OCP is written there:
 * N trays (tray 1 the condenser, tray N the reboiler), feed tray N_f, fixed
 * distillate flow D, reflux ratio u as the control, and the algebraic vapour
 * fractions y and flows L = u D, V = L + D, S = L + F kept as variables with
 * their own equality rows; objective dt sum_k (x_1 - xbar)^2 + w_u (u - ubar)^2
 * with (xbar, ubar) the setpoint parameter. */
enum {
    NMPC_FAMILY_DISTILLATION = 1,
    NMPC_FAMILY_HEATED_PLATE = 2,
    NMPC_FAMILY_REFLUX_COLUMN = 3,
    NMPC_FAMILY_STAGE_MODEL = 4   /* a model of the stage-pattern front end, see nmpc_stage_model */
};

/* A problem given by the pattern of one stage (eq. 3: one algebraic pattern
 * evaluated at every discretization point, its derivatives derived once and
 * compiled into kernels).  Every stage k = 1..H holds ns = nx + nu + na
 * variables in the order [states | controls | algebraic] and rps = nx +
 * n_alg_rows equality rows: first one row per state, which may also involve
 * the previous stage's states (the measured state x0 at stage 1), linearly
 * with the constant coefficients prev_coef, then the algebraic rows, which
 * involve the stage's own variables only.  Each stage also has n_ineq_rows
 * inequality rows d(stage) <= 0 in its own variables (stage-major after all
 * equality rows).  The objective is a sum of one term per stage in the
 * stage's variables, the previous stage's controls (u_prev at stage 1), the
 * setpoint and the stage's trajectory value.  The Hessian of the Lagrangian
 * is given per stage by its lower pattern within the stage (w_rows >= w_cols)
 * and, for stages 2..H, by the entries between the stage's variables and the
 * previous stage's controls (wx_rows, wx_cols).  Bounds go in lb / ub.
 *
 * The three kernels (value/derivative evaluation, cold-start guess, parameter
 * contractions of the sensitivities) come in a gfx950 code object written for
 * this library's kernel descriptor by the stage-pattern front end; the
 * library loads it on the problem's device and launches them by name
 * (nmpc_stage_eval, nmpc_stage_guess, nmpc_stage_adj); the kernels act only
 * on instances whose descriptor carries their tag.  Every pointer is host
 * memory the library copies at nmpc_create_problem.  Parameters: x0 (nx),
 * setpoint (n_setpoint), traj (H values, read when uses_traj), u_prev (nu,
 * read only by the cold-start guess). */
typedef struct nmpc_stage_model {
    int32_t nx, nu, na;         /* states (>= 1), controls (1..16), algebraic variables per stage */
    int32_t n_alg_rows;         /* equality rows per stage after the nx state rows */
    int32_t n_setpoint;         /* setpoint entries */
    int32_t uses_traj;          /* 1: the objective or rows read one trajectory value per stage */
    const int32_t* row_ptr;     /* rps + 1: own-stage columns of each stage row ... */
    const int32_t* row_cols;    /* ... strictly ascending, in [0, ns); a state row holds its own state */
    const int32_t* prev_ptr;    /* rps + 1: previous-stage state columns of each row (state rows only) ... */
    const int32_t* prev_cols;   /* ... strictly ascending, in [0, nx) */
    const double* prev_coef;    /* their constant coefficients, finite and nonzero */
    int32_t n_ineq_rows;        /* inequality rows per stage */
    const int32_t* ineq_ptr;    /* n_ineq_rows + 1: own-stage columns of each inequality row ... */
    const int32_t* ineq_cols;   /* ... strictly ascending, in [0, ns) */
    int32_t nw;                 /* lower Hessian entries per stage */
    const int32_t* w_rows;      /* nw: (w_rows[e], w_cols[e]), w_rows[e] >= w_cols[e], in [0, ns), distinct */
    const int32_t* w_cols;
    int32_t nw_cross;           /* Hessian entries per stage with the previous stage's controls (stages 2..H) */
    const int32_t* wx_rows;     /* nw_cross: the stage's variable, in [0, ns) ... */
    const int32_t* wx_cols;     /* ... and the previous stage's control, in [0, nu); pairs distinct */
    const double* lb;           /* ns: variable bounds of every stage; -inf / +inf for none, lb < ub */
    const double* ub;
    const void* code_object;    /* the kernels' code object ... */
    uint64_t code_object_size;  /* ... and its size in bytes */
    uint64_t tag;               /* the tag the kernels were generated with (nonzero) */
    int64_t scratch_per_stage;  /* doubles of per-stage scratch the kernels accumulate into (>= 0); when
                                   > 0 the code object also exports nmpc_stage_reduce, which the library
                                   launches after every evaluation to sum the scratch into the Hessian,
                                   gradient and objective terms; the library owns the array */
} nmpc_stage_model;

/* Fill-reducing ordering of the analysis (eq. 19).  NESTED_DISSECTION, the
 * default: stage-and-graph nested dissection of every family (boxes of stages
 * x stage variables cut by a middle stage or by one breadth-first level of the
 * graph the condensed matrix induces on a stage's states; controls and other
 * non-states follow their state neighbours' side, else the separator).
 * MIN_DEGREE: exact minimum degree of the condensed matrix's elimination
 * graph.  FAMILY_DISSECTION: the families' own dissections (one-stage
 * separators for the columns and front-end models, stage x grid slabs for the
 * plate). */
enum { NMPC_ORDER_NESTED_DISSECTION = 0, NMPC_ORDER_MIN_DEGREE = 1, NMPC_ORDER_FAMILY_DISSECTION = 2 };

/* How the Newton system of Section 3.2 is made solvable by Cholesky (the two
 * reformulations the section names).  LIFTED: Lifted-KKT, the equalities
 * relaxed to |c| <= gamma and lifted into inequalities (eq. 16); the condensed
 * matrix of eq. (17) is factored once per attempt.  HYKKT: the equalities kept
 * exact; the condensed system of eq. (14) with its equality block is solved by
 * the Cholesky factor of K_c + hykkt_gamma J_c^T J_c (same sparsity pattern
 * and symbolic analysis) and conjugate gradients on the Schur complement
 * J_c (K_c + hykkt_gamma J_c^T J_c)^{-1} J_c^T, one forward/back solve per CG
 * iteration.  The iterate converges to the original problem's KKT point
 * (no O(gamma) relaxation). */
enum { NMPC_KKT_LIFTED = 0, NMPC_KKT_HYKKT = 1 };

/* Problem structure: everything that fixes the sparsity pattern of the
 * transcribed OCP (eq. 6) and its constant data.  Parameters that change
 * between re-solves (x0, setpoints, disturbance trajectories, last control) go
 * through nmpc_set_parameters instead. */
typedef struct nmpc_structure {
    int32_t family;      /* NMPC_FAMILY_* */
    int32_t horizon;     /* H: number of implicit-Euler stages */
    double dt;           /* stage length */
    /* distillation column (Section 4.1 family) */
    int32_t n_trays;     /* N trays; states per stage N + 2, controls (R, V) */
    double alpha;        /* constant relative volatility */
    double feed_flow;    /* F */
    double move_penalty; /* rho on |u_k - u_{k-1}|^2 */
    double x_lo, x_hi;   /* mole-fraction bounds */
    double u_lo, u_hi;   /* bounds on R and V */
    /* heated plate (Section 4.2 family): G x G interior nodes (G a multiple of 4),
     * 16 Dirichlet heater segments (4 per edge), conductivity 1 + cond_slope T
     * averaged over each face, tracking objective sum_k sum_p (T_kp - T*_p)^2 */
    int32_t grid;        /* G */
    double t_hi;         /* upper temperature bound */
    double c_lo, c_hi;   /* heater control bounds */
    double cond_slope;   /* conductivity slope */
    int32_t ordering;    /* NMPC_ORDER_* */
    /* control horizon t_c <= t_p (Section 3.1, eqs. 4-5), distillation family:
     * with 1 <= control_horizon < horizon the controls of the stages after it
     * are held at its value, as equality rows u_k - u_{k-1} = 0 (the same
     * feasible set as u_k = u_{control_horizon}) placed after the dynamics
     * rows, R then V per stage; 0 (or >= horizon): every stage has its own
     * control.  The plate family must leave it 0. */
    int32_t control_horizon;
    /* reflux column (REFLUX_COLUMN; also uses n_trays, horizon, dt, alpha,
     * feed_flow, x_lo/x_hi for x and y, u_lo/u_hi for the reflux ratio):
     * feed tray (1-based), distillate flow D, feed composition x_f, molar
     * holdups of condenser, trays and reboiler, weight of (u - ubar)^2, upper
     * bound of the flows L, V, S (lower bound 0) */
    int32_t feed_tray;
    double distillate, feed_comp, hold_cond, hold_tray, hold_reb, u_weight, flow_hi;
    /* STAGE_MODEL: the stage pattern (also uses horizon, dt, ordering; the
     * control horizon must be 0) */
    const nmpc_stage_model* stage_model;
} nmpc_structure;

/* Interior-point constants (the paper leaves them open; see the design notes).
 * nmpc_default_options fills the defaults. */
typedef struct nmpc_options {
    double tol;          /* epsilon_outer on E_0, eq. (28) */
    double gamma;        /* equality relaxation of the lifting, eq. (16) */
    double mu0_cold, mu0_warm, mu_min;
    double kappa_eps;    /* inner test E_mu <= kappa_eps * mu, eq. (27) */
    double kappa_mu, theta_mu;
    double tau_min;      /* fraction-to-boundary */
    double armijo;
    int32_t ls_max;
    int32_t max_iter;
    double kappa_sigma;
    double eta_first, eta_min, eta_max, kp_first, kp, km;
    double bound_push, slack_push;
    /* filter line search (eq. 26 step, filter method of the cited interior-point
     * reference): sufficient-decrease margins gamma_theta, gamma_phi; switching
     * exponents s_theta, s_phi and factor delta; minimal step as a fraction of
     * the switching bound; theta_max / theta_min as factors of the first
     * iterate's violation; at most filter_cap entries (oldest dropped) */
    double filter_gamma_theta, filter_gamma_phi, filter_s_theta, filter_s_phi, filter_delta;
    double alpha_min_frac, theta_max_fact, theta_min_fact;
    int32_t filter_cap;
    /* second-order corrections of a rejected first trial point: at most soc_max,
     * each must reduce the violation by the factor soc_kappa (0 disables them) */
    int32_t soc_max;
    double soc_kappa;
    /* 1 (default): when the filter rejects every trial point down to the minimal
     * step, backtrack once more from the fraction-to-boundary step on the l1
     * merit phi + nu theta (Armijo; nu >= max |omega + d_omega| + 1, never
     * decreased within a solve), empty the filter on acceptance; 0: end the
     * solve with NMPC_LINESEARCH_FAIL there */
    int32_t merit_fallback;
    int32_t timing;      /* 1: record HIP events around each phase (device times in nmpc_result) */
    int32_t graph;       /* 1 (default): capture one pass of the method as a HIP graph and replay it;
                            0: launch every kernel of every pass from the host */
    int32_t fixed_mu;    /* 0 (default): Algorithm 2's barrier homotopy.  1: Newton's method on one
                            barrier problem: mu stays at its initial value (mu0_warm / mu0_cold), and
                            the solve ends when E_mu <= tol (eq. 27's inner test with tol in place
                            of kappa_eps mu), e.g. to re-solve a barrier solution tightly */
    /* NMPC_KKT_* (default LIFTED).  HYKKT runs nmpc_solve only (not batches),
     * launches its kernels from the host (graph ignored: the conjugate
     * gradients take one host round trip per iteration) and uses no
     * second-order corrections (soc_max ignored).  A warm HYKKT solve starts
     * from a held Lifted-KKT iterate too (lambda = omega+ - omega-); a warm
     * LIFTED solve from a HyKKT iterate is refused (BAD_ORDER), as are the
     * sensitivities of a HyKKT solution. */
    int32_t kkt;
    double hykkt_gamma;  /* weight of J_c^T J_c in the HyKKT matrix (default 1e6) */
    double hykkt_cg_tol; /* CG ends at |r|_2 <= hykkt_cg_tol |r_0|_2 (default 1e-12) */
    int32_t hykkt_cg_max;/* CG iterations per solve (default 200) */
} nmpc_options;

typedef struct nmpc_result {
    int32_t status;      /* NMPC_OK or a positive outcome */
    int32_t iters;       /* Newton iterations */
    int32_t factorizations;
    int32_t ls_trials;
    double mu, eta, E0, objective;
    double ms_total;     /* host wall time of the call */
    double ms_eval, ms_assemble, ms_factor, ms_solve, ms_linesearch; /* device phase times (0 unless timing enabled) */
    int32_t factor_launches; /* kernel launches spent in numeric factorizations */
    int32_t passes;      /* passes enqueued: one per Newton iteration, plus one per extra
                            factorization attempt or trial point (of the slowest instance of a batch) */
    int32_t timing_lost; /* passes whose phase times could not be read (then left out of ms_*) */
    int32_t cg_iters;    /* HyKKT: conjugate-gradient iterations over the solve (0 for LIFTED) */
} nmpc_result;

typedef struct nmpc_problem nmpc_problem;

/* Default interior-point options. */
void nmpc_default_options(nmpc_options* o);

/* Create a problem handle for a transcribed OCP family (eq. 6).  *s is copied;
 * the caller keeps ownership.  Builds the fixed Jacobian/Hessian/KKT patterns
 * on the host.  Needs no GPU.  Errors: INVALID_ARG for bad sizes/family. */
nmpc_status nmpc_create_problem(const nmpc_structure* s, nmpc_problem** out);

/* Release the handle and every host/device buffer it owns.  NULL is a no-op. */
void nmpc_destroy(nmpc_problem* p);

/* Sizes of the transcription: n variables, m_c dynamics rows, m_d inequality
 * rows, nx states and nu controls per stage, nnz of the lower KKT pattern. */
nmpc_status nmpc_sizes(const nmpc_problem* p, int32_t* n, int32_t* m_c, int32_t* m_d,
                       int32_t* nx, int32_t* nu, int64_t* nnz_k);

/* SymCholesky (eqs. 18-19): ordering, elimination tree, column counts,
 * supernodes and all scatter maps, computed once on the host and uploaded to
 * the device when one is present.  Idempotent: a second call is a no-op. */
nmpc_status nmpc_analyze(nmpc_problem* p);

/* Sizes of the symbolic analysis: supernode count, stored entries of the
 * supernodal factor (explicit zeros included), exact nnz(L) and sum of
 * squared column counts, total supernode row-list length, etree depth in
 * supernodes.  BAD_ORDER before nmpc_analyze. */
nmpc_status nmpc_symbolic_sizes(const nmpc_problem* p, int32_t* n_supernodes, int64_t* stored_l,
                                int64_t* nnz_l, int64_t* flops, int64_t* rows_total, int32_t* depth);

/* Export the symbolic analysis into caller-allocated host arrays (any may be
 * NULL): perm[n] (new -> old), parent[n] (column etree in the final order,
 * -1 for roots), colcount[n], snode_ptr[n_supernodes + 1],
 * snode_rows_ptr[n_supernodes + 1] (int64) and snode_rows[rows_total]
 * (sorted row indices of each supernode, its own columns first). */
nmpc_status nmpc_export_symbolic(const nmpc_problem* p, int32_t* perm, int32_t* parent,
                                 int32_t* colcount, int32_t* snode_ptr,
                                 int64_t* snode_rows_ptr, int32_t* snode_rows);

/* Export the structural patterns (host, caller-allocated, any may be NULL):
 * Jacobian rows/cols of [c; d] (nnz_j entries, original variable order),
 * lower Hessian rows/cols (nnz_w entries), lower KKT rows/cols (nnz_k
 * entries, original order, in the library's slot order). */
nmpc_status nmpc_pattern_sizes(const nmpc_problem* p, int64_t* nnz_j, int64_t* nnz_w, int64_t* nnz_k);
nmpc_status nmpc_export_patterns(const nmpc_problem* p, int32_t* j_rows, int32_t* j_cols,
                                 int32_t* w_rows, int32_t* w_cols, int32_t* k_rows, int32_t* k_cols);

/* Parameters p_k of the next solve (eq. 4), host arrays copied before return:
 * x0[nx] measured initial state; setpoint: distillation (xD*, xB*), plate
 * target field [G*G] (NULL keeps the previous one); traj: distillation feed
 * composition zF[H] (NULL keeps the previous one; the plate has none);
 * u_prev[nu]: control applied before stage 1 (NULL keeps the previous one; the
 * plate uses it only for the cold-start guess).  Errors: INVALID_ARG on NULL
 * x0 or non-finite values. */
nmpc_status nmpc_set_parameters(nmpc_problem* p, const double* x0, const double* setpoint,
                                const double* traj, const double* u_prev);

/* One NMPC solve (Algorithm 2).  warm = 0: cold start from x0 repeated over
 * the horizon with u_prev, mu = mu0_cold.  warm = 1: start from the last
 * iterate held by the handle (Algorithm 1, z_{k+1} <- z*_k) with mu0_warm.
 * warm = 2: the same, shifted by one stage first (stage k takes stage k + 1's
 * values of every stage-indexed quantity, the last stage keeps its own: the
 * horizon has advanced by one stage since that solution).  An arbitrary
 * warm start is placed with nmpc_set_iterate, then warm = 1.
 * opts NULL = defaults.  res may be NULL.  Returns NMPC_OK, a positive
 * outcome, or an error (BAD_ORDER before analyze or warm without a previous
 * solve; NO_DEVICE without a GPU). */
nmpc_status nmpc_solve(nmpc_problem* p, int32_t warm, const nmpc_options* opts, nmpc_result* res);

/* Copy the last iterate to host arrays (any may be NULL): y[n], lam[m_c]
 * (equality multipliers omega+ - omega-), omega_d[m_d], zL[n], zU[n],
 * u1[nu] (first-stage control, Algorithm 1 line "extract"), x1[nx]. */
nmpc_status nmpc_get_solution(const nmpc_problem* p, double* y, double* lam, double* omega_d,
                              double* zL, double* zU, double* u1, double* x1);

/* Full primal-dual iterate z = (y, s, omega, beta, zL, zU) with the lifted
 * vectors of length m^l = 2 m_c + m_d ordered [plus rows, minus rows, d rows].
 * get copies it out; set replaces the handle's iterate (a warm start from an
 * arbitrary point).  Host arrays, none may be NULL. */
nmpc_status nmpc_get_iterate(const nmpc_problem* p, double* y, double* s, double* omega,
                             double* beta, double* zL, double* zU);
nmpc_status nmpc_set_iterate(nmpc_problem* p, const double* y, const double* s, const double* omega,
                             const double* beta, const double* zL, const double* zU);

/* Model evaluation on the device (eqs. 3, 11): at y[n] with equality
 * multipliers lam[m_c] and inequality multipliers lam_d[m_d], return f,
 * grad[n], c[m_c], d[m_d], Jacobian values j_vals[nnz_j] and lower Hessian of
 * the Lagrangian w_vals[nnz_w], in the slot order nmpc_export_patterns gives.
 * Host arrays; outputs may be NULL. */
nmpc_status nmpc_eval(nmpc_problem* p, const double* y, const double* lam, const double* lam_d,
                      double* f, double* grad, double* c, double* d, double* j_vals, double* w_vals);

/* NumCholesky (eqs. 20-21) of a caller-given matrix: k_vals[nnz_k] are the
 * lower KKT values in slot order; eta is added to the diagonal.  On return
 * *ok = 1 when every pivot was positive and finite.  l_vals (may be NULL)
 * receives the supernodal factor: for supernode s, a column-major
 * rows(s) x width(s) panel, panels in supernode order (stored_l values).
 * Requires nmpc_analyze. */
nmpc_status nmpc_factor(nmpc_problem* p, const double* k_vals, double eta, int32_t* ok,
                        double* l_vals);

/* Forward/back substitution with the factor of the last nmpc_factor or
 * iteration (eqs. 22-25): solves K x = b, b and x in the original order. */
nmpc_status nmpc_linear_solve(nmpc_problem* p, const double* b, double* x);

/* Condensed assembly (eqs. 14, 17) at the handle's current iterate and mu:
 * returns the lower KKT values without regularization and the right-hand
 * side -r1 - G^T (Q r4 - r2). */
nmpc_status nmpc_assemble(nmpc_problem* p, double mu, double* k_vals, double* rhs);

/* Sensitivities of the last solution: the lifted barrier KKT conditions of
 * Section 3.2 (eqs. 8-9 for the lifted problem of eq. 16) are differentiated by
 * the implicit function theorem and condensed as in eqs. (14) and (17), so
 * K dy/dp = -d(grad f)/dp - J_c^T (Q+ + Q-) dc/dp - J_d^T Q_d dd/dp with K the
 * condensed matrix at the returned iterate.  K is assembled and factored once
 * (kept until the next solve, iterate or parameter change) and reused by every
 * call; one forward/back solve per seed.
 * nmpc_adjoint: gradient of seed_u1 . u1* + seed_obj * f* (vector-Jacobian
 * product) with respect to x0 (grad_x0[nx]), the setpoint (grad_setpoint:
 * distillation (xD*, xB*), plate the target field [G*G]), the disturbance
 * trajectory (grad_traj: distillation zF[H]; untouched for the plate) and
 * u_prev (grad_uprev[nu]; zeros for the plate); outputs may be NULL, seed_u1
 * may not.  Host arrays.
 * BAD_ORDER without a solution or when parameters were set after it;
 * REG_FAIL (positive) when K needed eta > 0 to factor (the gradient is then
 * that of the regularized system). */
nmpc_status nmpc_adjoint(nmpc_problem* p, const double* seed_u1, double seed_obj, double* grad_x0,
                         double* grad_setpoint, double* grad_traj, double* grad_uprev);

/* Jacobian d u1* / d x0 as an nu x nx row-major host matrix: row k is the
 * x0 gradient nmpc_adjoint returns for seed_u1 = e_k, seed_obj = 0 (the same
 * arithmetic).  The nu seeds are solved together with the kept factor, every
 * launch covering all of them; the first call after analysis allocates their
 * vectors (about 8 (5 n + 2 m + update vectors) bytes per seed), later calls
 * reuse them.  Same conditions as nmpc_adjoint. */
nmpc_status nmpc_jacobian_u1_x0(nmpc_problem* p, double* jac);

/* Allocation-free variant of nmpc_jacobian_u1_x0, for callers that cannot
 * allocate device memory while they call it (code under HIP stream capture,
 * tight serving loops, harnesses that forbid hipMalloc).  It allocates nothing
 * (no hipMalloc, hipFree or allocating library call) on any call: the nu seeds
 * are solved one after another, each with the same kernels and refinement as
 * nmpc_jacobian_u1_x0, and the vectors they write live in one fixed device
 * buffer of NMPC_NOALLOC_SCRATCH_BYTES per GPU, which the library holds from
 * its first use on that GPU until the process ends.
 * jac: device pointer, nu x nx row-major, owned by the caller; stream: the
 * caller's hipStream_t (NULL = the null stream), ordered as the *_dev entry
 * points below.  Every call on one GPU shares that GPU's buffer and the
 * buffer keeps the last call's contents (a call writes everything it reads
 * there before reading it), so calls that overlap on one GPU race (two host
 * threads, or two streams whose work can overlap): serialize them.  The first
 * sensitivity call after a solve factors K at the solution and waits for the
 * library's stream once.
 * Errors: UNSUPPORTED when the problem needs more of the buffer than there is
 * (about 8 (6 n + 2 m + update-vector entries) bytes; the 64 x 64 x 100 plate
 * needs 91 MiB), then use nmpc_jacobian_u1_x0; otherwise as
 * nmpc_jacobian_u1_x0. */
#define NMPC_NOALLOC_SCRATCH_BYTES (128u * 1024u * 1024u)
nmpc_status nmpc_jacobian_u1_x0_noalloc(nmpc_problem* p, double* jac, void* stream);

/* Identity of the iterate the handle holds: *id counts the iterates it has
 * taken (each nmpc_solve that returned a status >= 0, each batch solve it was
 * part of, each nmpc_set_iterate; 0 before the first); *current (may be NULL)
 * is 1 while no parameter has been set since, 0 otherwise.  The
 * sensitivities differentiate the held iterate for the parameters it was
 * computed with, so nmpc_adjoint, nmpc_adjoint_dev and nmpc_jacobian_u1_x0
 * return BAD_ORDER when *current would be 0; a caller that differentiates
 * later (e.g. an autograd backward) compares *id with the one it saw after
 * its solve. */
nmpc_status nmpc_solution_id(const nmpc_problem* p, int64_t* id, int32_t* current);

/* Device-pointer variants (Algorithm 1's parameter update, the solution read
 * and the sensitivities without a host round trip, e.g. for tensors that live
 * on the GPU).  Every pointer is a device address on the handle's GPU, owned by
 * the caller; stream is a hipStream_t of the caller (NULL = the null stream).
 * The library's work waits for everything already enqueued on stream and the
 * work enqueued on stream afterwards waits for the library's, so buffers may
 * be reused in stream order; the calls do not synchronize the host.
 * Values are not checked on the host: a non-finite parameter shows up as the
 * solve's NMPC_NONFINITE.  Requires nmpc_analyze (BAD_ORDER otherwise).
 *
 * nmpc_set_parameters_dev: as nmpc_set_parameters (NULL keeps the previous
 *   setpoint / traj / u_prev; x0 may not be NULL).
 * nmpc_get_solution_dev: as nmpc_get_solution, into device buffers.
 * nmpc_adjoint_dev: as nmpc_adjoint; seed_u1[nu] and seed_obj (one value) are
 *   device pointers (NULL = zero).  The first sensitivity call after a solve
 *   factors K at the solution and waits for the library's stream once. */
nmpc_status nmpc_set_parameters_dev(nmpc_problem* p, const double* x0, const double* setpoint,
                                    const double* traj, const double* u_prev, void* stream);
nmpc_status nmpc_get_solution_dev(const nmpc_problem* p, double* y, double* lam, double* omega_d,
                                  double* zL, double* zU, double* u1, double* x1, void* stream);
nmpc_status nmpc_adjoint_dev(nmpc_problem* p, const double* seed_u1, const double* seed_obj, double* grad_x0,
                             double* grad_setpoint, double* grad_traj, double* grad_uprev, void* stream);

/* Closed loop on the device (Algorithm 1 with plant = model: the applied
 * control and the next measurement never leave the GPU).  Starting from the
 * held solution, for k = 0 .. steps-1: the solution's first stage is the
 * applied control u1 and the predicted state x1 (written to row k of u_out,
 * steps x nu, and of x_out, steps x nx, when not NULL); the next parameters
 * are formed on the device: x0 = x1 + noise row k (noise: steps x nx, NULL =
 * none), clipped to the first stage's state bounds; u_prev = u1; traj = row k
 * of traj (steps x H, NULL = kept); the setpoint is kept; then the problem is
 * re-solved warm (as nmpc_solve with warm = 1).  The parameter update, the
 * reset of the interior-point control block and passes_per_step passes of the
 * method are one captured graph, replayed once per step; the host then reads
 * two integers and replays single passes until the solve stops, so a step
 * costs one host round trip when it converges within passes_per_step passes.
 * Every pointer is a device address on the handle's GPU owned by the caller;
 * stream as for the _dev entry points.  Requires a held Lifted-KKT solution
 * for the current parameters (BAD_ORDER otherwise) and options with
 * kkt = NMPC_KKT_LIFTED and timing = 0 (INVALID_ARG otherwise);
 * 1 <= passes_per_step <= 16.  Returns NMPC_OK when every step's solve
 * succeeded, else the first failing solve's status (a positive outcome as
 * nmpc_solve's), with *steps_done the number of steps taken (the failing one
 * included) and *iters_total their interior-point iterations; the problem then
 * holds that step's iterate and parameters (host copies updated). */
nmpc_status nmpc_closed_loop_dev(nmpc_problem* p, int32_t steps, const double* traj, const double* noise,
                                 double* u_out, double* x_out, int32_t passes_per_step, const nmpc_options* opts,
                                 int32_t* steps_done, int32_t* iters_total, void* stream);

/* Autotuner of the supernode front kernels (the batched form's tile shapes):
 * for every factor launch of the problem's schedule, time each variant of the
 * one-workgroup front kernel (threads per workgroup 128 / 256 / 512, panel
 * width 4 / 8) on a diagonally dominant matrix with the problem's pattern and
 * keep the fastest; the symbolic partition is not changed.  Choices are cached
 * per structure hash for the life of the process, so problems of equal
 * structure are tuned once.  reps: timed repetitions per variant (>= 1);
 * *changed (may be NULL): launches whose variant is not the default.
 * Overwrites the held factor (sensitivities refactor).  Requires
 * nmpc_analyze and a device; call before nmpc_batch_create for a batch. */
nmpc_status nmpc_autotune(nmpc_problem* p, int32_t reps, int32_t* changed);

/* Batches (the batched form): several analyzed problems, of any sizes, solved
 * together.  Every kernel of a pass covers all instances at once (block ->
 * instance tables, one launch per level of the deepest supernodal schedule),
 * the method's decisions are taken per instance on the device, and an instance
 * that has converged idles while the others continue.  Each instance's
 * arithmetic is the same as in its own nmpc_solve.
 * nmpc_batch_create: problems[count] (distinct, analyzed, each with a device)
 * are referenced, not copied or owned: they must outlive the batch, and their
 * parameters are still set with nmpc_set_parameters.  Errors: INVALID_ARG
 * (NULL, count < 1, duplicates), BAD_ORDER (a problem not analyzed),
 * NO_DEVICE. */
typedef struct nmpc_batch nmpc_batch;
nmpc_status nmpc_batch_create(nmpc_problem* const* problems, int32_t count, nmpc_batch** out);
/* Solve every instance (Algorithm 2 per instance); warm as in nmpc_solve, for
 * all instances.  per_instance[count] (may be NULL) receives each instance's
 * result; the phase times are those of the whole batch.  Returns the largest
 * instance status, or an error.  Afterwards each problem's solution is read
 * with nmpc_get_solution. */
nmpc_status nmpc_batch_solve(nmpc_batch* b, int32_t warm, const nmpc_options* opts, nmpc_result* per_instance);
/* Release the batch (not its problems).  NULL is a no-op. */
void nmpc_batch_destroy(nmpc_batch* b);

/* Thread-local message for the last error on this thread. */
const char* nmpc_last_error(void);

/* 1 when a HIP device is visible, 0 otherwise. */
int32_t nmpc_device_available(void);

#ifdef __cplusplus
}
#endif
#endif /* NMPC_H */
