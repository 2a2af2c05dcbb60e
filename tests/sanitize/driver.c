/* Walks the host side of the C ABI (transcription, symbolic analysis, pattern
 * and symbolic export, parameter checks, error paths) under AddressSanitizer
 * and UndefinedBehaviorSanitizer, linked against a device layer that reports
 * no device.  Prints one line per case and "sanitize: ok" at the end; any
 * unexpected status exits non-zero.  Test infrastructure only. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "nmpc.h"

static int failures = 0;

#define EXPECT(cond, what)                                                       \
    do {                                                                         \
        if (!(cond)) {                                                           \
            fprintf(stderr, "FAILED: %s (%s) last error: %s\n", what, #cond,      \
                    nmpc_last_error());                                          \
            ++failures;                                                          \
        }                                                                        \
    } while (0)

static nmpc_structure distill(int N, int H, int ordering) {
    nmpc_structure s;
    memset(&s, 0, sizeof(s));
    s.family = NMPC_FAMILY_DISTILLATION;
    s.horizon = H;
    s.dt = 0.05;
    s.n_trays = N;
    s.alpha = 2.5;
    s.feed_flow = 1.0;
    s.move_penalty = 1e-2;
    s.x_lo = 0.0;
    s.x_hi = 1.0;
    s.u_lo = 0.5;
    s.u_hi = 5.0;
    s.ordering = ordering;
    return s;
}

static nmpc_structure plate(int G, int H, int ordering) {
    nmpc_structure s;
    memset(&s, 0, sizeof(s));
    s.family = NMPC_FAMILY_HEATED_PLATE;
    s.horizon = H;
    s.dt = 0.01;
    s.grid = G;
    s.t_hi = 1.5;
    s.c_lo = 0.0;
    s.c_hi = 1.0;
    s.cond_slope = 0.1;
    s.ordering = ordering;
    return s;
}

static void walk(const nmpc_structure* s, const char* name) {
    nmpc_problem* p = NULL;
    int32_t n = 0, mc = 0, md = 0, nx = 0, nu = 0;
    int64_t nnzk = 0, nnzj = 0, nnzw = 0, nnzk2 = 0;
    EXPECT(nmpc_create_problem(s, &p) == NMPC_OK && p, name);
    if (!p) return;
    EXPECT(nmpc_sizes(p, &n, &mc, &md, &nx, &nu, &nnzk) == NMPC_OK, name);
    EXPECT(nmpc_pattern_sizes(p, &nnzj, &nnzw, &nnzk2) == NMPC_OK && nnzk2 == nnzk, name);
    int32_t* jr = malloc(sizeof(int32_t) * (size_t)(nnzj + 1));
    int32_t* jc = malloc(sizeof(int32_t) * (size_t)(nnzj + 1));
    int32_t* wr = malloc(sizeof(int32_t) * (size_t)(nnzw + 1));
    int32_t* wc = malloc(sizeof(int32_t) * (size_t)(nnzw + 1));
    int32_t* kr = malloc(sizeof(int32_t) * (size_t)(nnzk + 1));
    int32_t* kc = malloc(sizeof(int32_t) * (size_t)(nnzk + 1));
    EXPECT(nmpc_export_patterns(p, jr, jc, wr, wc, NULL, NULL) == NMPC_OK, name);
    /* KKT slot order exists only after the analysis */
    EXPECT(nmpc_export_patterns(p, NULL, NULL, NULL, NULL, kr, kc) == NMPC_ERR_BAD_ORDER, name);
    EXPECT(nmpc_solve(p, 0, NULL, NULL) == NMPC_ERR_BAD_ORDER, name);
    EXPECT(nmpc_symbolic_sizes(p, NULL, NULL, NULL, NULL, NULL, NULL) == NMPC_ERR_BAD_ORDER, name);
    EXPECT(nmpc_analyze(p) == NMPC_OK, name);
    EXPECT(nmpc_analyze(p) == NMPC_OK, name); /* idempotent */
    EXPECT(nmpc_export_patterns(p, NULL, NULL, NULL, NULL, kr, kc) == NMPC_OK, name);
    int32_t nsn = 0, depth = 0;
    int64_t stored = 0, nnzl = 0, flops = 0, rows = 0;
    EXPECT(nmpc_symbolic_sizes(p, &nsn, &stored, &nnzl, &flops, &rows, &depth) == NMPC_OK, name);
    EXPECT(nsn > 0 && stored >= nnzl && nnzl >= n && rows > 0 && depth > 0, name);
    int32_t* perm = malloc(sizeof(int32_t) * (size_t)n);
    int32_t* parent = malloc(sizeof(int32_t) * (size_t)n);
    int32_t* cc = malloc(sizeof(int32_t) * (size_t)n);
    int32_t* sptr = malloc(sizeof(int32_t) * (size_t)(nsn + 1));
    int64_t* rptr = malloc(sizeof(int64_t) * (size_t)(nsn + 1));
    int32_t* srows = malloc(sizeof(int32_t) * (size_t)rows);
    EXPECT(nmpc_export_symbolic(p, perm, parent, cc, sptr, rptr, srows) == NMPC_OK, name);
    /* perm is a permutation; the etree points forward; supernodes tile the columns */
    char* seen = calloc((size_t)n, 1);
    int ok = 1;
    for (int i = 0; i < n; ++i) {
        if (perm[i] < 0 || perm[i] >= n || seen[perm[i]]) ok = 0;
        else seen[perm[i]] = 1;
        if (parent[i] != -1 && parent[i] <= i) ok = 0;
    }
    ok = ok && sptr[0] == 0 && sptr[nsn] == n && rptr[0] == 0 && rptr[nsn] == rows;
    EXPECT(ok, name);
    /* parameters: sizes from the structure; non-finite values refused */
    double* x0 = malloc(sizeof(double) * (size_t)nx);
    for (int i = 0; i < nx; ++i) x0[i] = 0.5;
    double up[16];
    for (int i = 0; i < 16; ++i) up[i] = 1.0;
    EXPECT(nmpc_set_parameters(p, x0, NULL, NULL, up) == NMPC_OK, name);
    x0[nx / 2] = NAN;
    EXPECT(nmpc_set_parameters(p, x0, NULL, NULL, NULL) == NMPC_ERR_INVALID_ARG, name);
    EXPECT(nmpc_set_parameters(p, NULL, NULL, NULL, NULL) == NMPC_ERR_INVALID_ARG, name);
    /* everything numeric needs the device */
    EXPECT(nmpc_solve(p, 0, NULL, NULL) == NMPC_ERR_NO_DEVICE, name);
    double seed[16] = {0};
    EXPECT(nmpc_adjoint(p, seed, 1.0, NULL, NULL, NULL, NULL) == NMPC_ERR_BAD_ORDER, name);
    EXPECT(nmpc_adjoint(p, NULL, 1.0, NULL, NULL, NULL, NULL) == NMPC_ERR_INVALID_ARG, name);
    int64_t sid = -1;
    int32_t cur = -1;
    EXPECT(nmpc_solution_id(p, &sid, &cur) == NMPC_OK && sid == 0 && cur == 0, name);
    EXPECT(nmpc_autotune(p, 1, NULL) == NMPC_ERR_NO_DEVICE, name);
    nmpc_batch* b = NULL;
    EXPECT(nmpc_batch_create(&p, 1, &b) == NMPC_ERR_NO_DEVICE && b == NULL, name);
    printf("%s: n %d m_c %d m_d %d nnz_k %lld supernodes %d nnz_l %lld depth %d\n", name, n, mc, md,
           (long long)nnzk, nsn, (long long)nnzl, depth);
    free(seen); free(x0); free(perm); free(parent); free(cc); free(sptr); free(rptr); free(srows);
    free(jr); free(jc); free(wr); free(wc); free(kr); free(kc);
    nmpc_destroy(p);
}

int main(void) {
    nmpc_options o;
    nmpc_default_options(&o);
    EXPECT(o.tol > 0 && o.graph == 1 && o.fixed_mu == 0, "defaults");
    EXPECT(nmpc_device_available() == 0, "no device");
    nmpc_problem* p = NULL;
    EXPECT(nmpc_create_problem(NULL, &p) == NMPC_ERR_INVALID_ARG, "NULL structure");
    nmpc_structure bad = distill(10, 20, 0);
    bad.horizon = 0;
    EXPECT(nmpc_create_problem(&bad, &p) == NMPC_ERR_INVALID_ARG && p == NULL, "horizon 0");
    bad = plate(10, 3, 0);   /* G not a multiple of 4 */
    EXPECT(nmpc_create_problem(&bad, &p) == NMPC_ERR_INVALID_ARG && p == NULL, "grid 10");
    bad = distill(1, 20, 0);   /* fewer than two trays */
    EXPECT(nmpc_create_problem(&bad, &p) == NMPC_ERR_INVALID_ARG && p == NULL, "one tray");
    bad = distill(10, 20, 0);
    bad.family = 99;
    EXPECT(nmpc_create_problem(&bad, &p) == NMPC_ERR_UNSUPPORTED && p == NULL, "family 99");
    EXPECT(nmpc_batch_create(NULL, 0, NULL) == NMPC_ERR_INVALID_ARG, "batch NULL");
    nmpc_destroy(NULL);
    nmpc_batch_destroy(NULL);
    for (int ord = 0; ord < 2; ++ord) {
        nmpc_structure s = distill(10, 20, ord);
        walk(&s, ord ? "distillation 10x20 min-degree" : "distillation 10x20");
        s = distill(2, 1, ord);
        walk(&s, ord ? "distillation 2x1 min-degree" : "distillation 2x1");
        s = plate(8, 3, ord);
        walk(&s, ord ? "plate 8x8x3 min-degree" : "plate 8x8x3");
    }
    nmpc_structure s = distill(40, 100, 0);
    walk(&s, "distillation 40x100");
    s = plate(16, 10, 0);
    walk(&s, "plate 16x16x10");
    if (failures) {
        fprintf(stderr, "sanitize: %d failure(s)\n", failures);
        return 1;
    }
    printf("sanitize: ok\n");
    return 0;
}
