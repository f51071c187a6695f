/*
 * Driver of the sanitizer build (tests/test_sanitizers.py): the oracle
 * (oracle/wto_oracle.c) and the host build of the kernels' arithmetic
 * (paper_1504_00731_amd/csrc/host_check.cpp) compiled with AddressSanitizer and
 * UndefinedBehaviorSanitizer, run over the boundary conditions, side tables,
 * dimensions and error paths, so that an out-of-bounds stencil or ghost index, a
 * leak or undefined arithmetic aborts the run.  The two are only called here;
 * they share no code.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "wto_oracle.h"

/* host_check.cpp */
int wth_rhs(int prec, int sys, int ndim, const int64_t *n, const double *dx, const int *bc,
            const double *alpha, double gamma, double eps, double aR, const double *u,
            const double *f, double *L, const double *grav);
int64_t wth_map_index(int64_t i, int64_t n, int bc);
int wth_reflected(int64_t i, int64_t n, int bc);

static uint64_t rng_state = 12345u;

static double urand(void)
{
    rng_state = rng_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(rng_state >> 11) * 0x1p-53;
}

/* A random physical Euler state (rho in [0.5, 1.5], |v| <= 0.5, p in [0.5, 1.5]). */
static void random_state(int ndim, int64_t N, double *u)
{
    for (int64_t j = 0; j < N; ++j) {
        const double rho = 0.5 + urand();
        double v2 = 0.0;
        for (int d = 0; d < ndim; ++d) {
            const double v = urand() - 0.5;
            u[(1 + d) * N + j] = rho * v;
            v2 += v * v;
        }
        u[j] = rho;
        u[(ndim + 1) * N + j] = (0.5 + urand()) / 0.4 + 0.5 * rho * v2;
    }
}

static int failures = 0;

static void check(int ok, const char *what)
{
    if (!ok) {
        fprintf(stderr, "FAILED: %s\n", what);
        ++failures;
    }
}

static wto_problem euler(int ndim, const int64_t *n, int bc)
{
    wto_problem P;
    memset(&P, 0, sizeof P);
    P.ndim = ndim;
    P.system = WTO_EULER;
    for (int k = 0; k < 3; ++k) {
        P.n[k] = k < ndim ? n[k] : 1;
        P.dx[k] = k < ndim ? 1.0 / (double)n[k] : 1.0;
        P.bc[k] = k < ndim ? bc : WTO_PERIODIC;
    }
    P.gamma = 1.4;
    P.cfl = 0.5;
    P.eps = 1e-10;
    P.alpha_R = 50.0;
    return P;
}

/* RHS and two steps of the oracle; the host build's RHS on the same state. */
static void run_case(wto_problem *P, const char *what)
{
    const int m = P->system == WTO_EULER ? P->ndim + 2 : 1;
    const int64_t N = P->n[0] * P->n[1] * P->n[2];
    double *u = malloc(sizeof(double) * m * N), *L = malloc(sizeof(double) * m * N);
    double *L2 = malloc(sizeof(double) * m * N);
    random_state(P->ndim, N, u);
    check(wto_rhs(P, u, NULL, NULL, L) == WTO_OK, what);
    double alpha[15], amax[3];
    check(wto_alpha(P, u, alpha, amax) == WTO_OK, what);
    if (P->bc[0] != WTO_SIDES && P->bc[1] != WTO_SIDES && P->bc[2] != WTO_SIDES) {
        double al[15] = {0};
        for (int d = 0; d < P->ndim; ++d)
            for (int s = 0; s < m; ++s) al[d * 5 + s] = alpha[d * m + s];
        const int bc[3] = {P->bc[0], P->bc[1], P->bc[2]};
        for (int prec = 0; prec < 3; ++prec)
            check(wth_rhs(prec, WTO_EULER, P->ndim, P->n, P->dx, bc, al, P->gamma, P->eps,
                          P->alpha_R, u, NULL, L2, P->gravity) == 0, what);
    }
    for (int d = 0; d < P->ndim; ++d) {
        int64_t ext = 1;
        for (int k = 0; k < 3; ++k) ext *= k == d ? P->n[k] + 1 : P->n[k];
        int32_t *dec = malloc(sizeof(int32_t) * ext * m * 4);
        double *mar = malloc(sizeof(double) * ext * m * 4);
        check(wto_decisions(P, u, NULL, d, dec, mar) == WTO_OK, what);
        free(dec);
        free(mar);
    }
    double dt = 0.0;
    for (int k = 0; k < 2; ++k) check(wto_step(P, u, 0.0, &dt) == WTO_OK, what);
    free(u);
    free(L);
    free(L2);
}

int main(void)
{
    /* 1D, 2D, 3D with every plain boundary condition, short and ragged lines */
    const int bcs[3] = {WTO_PERIODIC, WTO_TRANSMISSIVE, WTO_REFLECTIVE};
    for (int b = 0; b < 3; ++b) {
        const int64_t n1[1] = {6}, n1b[1] = {37}, n2[2] = {7, 6}, n3[3] = {6, 7, 8};
        wto_problem P;
        P = euler(1, n1, bcs[b]); run_case(&P, "1D n=6");
        P = euler(1, n1b, bcs[b]); run_case(&P, "1D n=37");
        P = euler(2, n2, bcs[b]); run_case(&P, "2D 7x6");
        P = euler(3, n3, bcs[b]); run_case(&P, "3D 6x7x8");
    }
    /* gravity with walls */
    {
        const int64_t n2[2] = {9, 12};
        wto_problem P = euler(2, n2, WTO_REFLECTIVE);
        P.gravity[1] = 0.1;
        run_case(&P, "2D walls + gravity");
    }
    /* side tables: given states, walls and zero gradient split at moving points */
    {
        const int64_t n2[2] = {12, 9}, n3[3] = {7, 6, 8};
        wto_side sides[6];
        memset(sides, 0, sizeof sides);
        for (int i = 0; i < 6; ++i) {
            sides[i].kind[0] = i % 3 == 0 ? WTO_STATE : WTO_REFLECTIVE;
            sides[i].kind[1] = i % 2 == 0 ? WTO_TRANSMISSIVE : WTO_STATE;
            for (int q = 0; q < 2; ++q) sides[i].state[q][0] = 1.0 + 0.1 * q;
            sides[i].split0 = 0.3 + 0.05 * i;
            sides[i].split_speed = 2.0;
        }
        /* given states (rho, m.., E) with ndim momentum entries */
        for (int ndim = 1; ndim <= 3; ++ndim) {
            for (int i = 0; i < 6; ++i)
                for (int q = 0; q < 2; ++q) {
                    for (int c = 1; c <= ndim; ++c) sides[i].state[q][c] = 0.1 / c;
                    sides[i].state[q][ndim + 1] = 2.5 + 0.1 * q;
                    for (int c = ndim + 2; c < 5; ++c) sides[i].state[q][c] = 0.0;
                }
            const int64_t n1[1] = {10};
            wto_problem P = ndim == 1 ? euler(1, n1, WTO_SIDES)
                                      : (ndim == 2 ? euler(2, n2, WTO_SIDES) : euler(3, n3, WTO_SIDES));
            P.sides = sides;
            P.t = 0.01;
            run_case(&P, ndim == 1 ? "1D sides" : (ndim == 2 ? "2D sides" : "3D sides"));
        }
    }
    /* scalar laws: RHS with caller flux values, solve, decisions */
    {
        wto_problem P;
        memset(&P, 0, sizeof P);
        P.ndim = 1;
        P.system = WTO_BURGERS;
        P.n[0] = 50; P.n[1] = P.n[2] = 1;
        P.dx[0] = 0.04; P.dx[1] = P.dx[2] = 1.0;
        P.bc[0] = WTO_TRANSMISSIVE;
        P.cfl = 0.5; P.eps = 1e-10; P.alpha_R = 50.0; P.gamma = 1.4;
        double u[50], f[50], L[50], al = 0.0;
        for (int j = 0; j < 50; ++j) {
            u[j] = sin(0.3 * j);
            f[j] = 0.5 * u[j] * u[j];
            if (fabs(u[j]) > al) al = fabs(u[j]);
        }
        check(wto_rhs(&P, u, f, &al, L) == WTO_OK, "burgers rhs");
        double t = 0.0;
        int64_t k = 0;
        check(wto_solve(&P, u, 0.0, 0.5, -1, &t, &k) == WTO_OK, "burgers solve");
        int32_t dec[51 * 4];
        double mar[51 * 4];
        check(wto_decisions(&P, u, NULL, 0, dec, mar) == WTO_OK, "burgers decisions");
        const int64_t n[3] = {50, 1, 1};
        const double dx[3] = {0.04, 1.0, 1.0};
        const int bc[3] = {WTO_TRANSMISSIVE, 0, 0};
        const double a5[15] = {al};
        for (int prec = 0; prec < 3; ++prec)
            check(wth_rhs(prec, WTO_BURGERS, 1, n, dx, bc, a5, 1.4, 1e-10, 50.0, u, f, L, NULL) == 0,
                  "burgers host rhs");
    }
    /* error paths: a non-physical state is reported, not read past */
    {
        const int64_t n2[2] = {8, 8};
        wto_problem P = euler(2, n2, WTO_TRANSMISSIVE);
        double *u = malloc(sizeof(double) * 4 * 64), *L = malloc(sizeof(double) * 4 * 64);
        random_state(2, 64, u);
        u[3 * 64 + 10] = -1.0;
        check(wto_rhs(&P, u, NULL, NULL, L) == WTO_ERR_NONPHYSICAL, "non-physical reported");
        free(u);
        free(L);
    }
    /* boundary index maps far outside short lines */
    for (int64_t n = 6; n < 40; ++n)
        for (int b = 0; b < 3; ++b)
            for (int64_t i = -600; i < n + 600; ++i) {
                const int64_t j = wth_map_index(i, n, bcs[b]);
                check(j >= 0 && j < n, "map index in range");
                (void)wth_reflected(i, n, bcs[b]);
            }
    if (failures) {
        fprintf(stderr, "%d failures\n", failures);
        return 1;
    }
    printf("sanitized runs ok\n");
    return 0;
}
