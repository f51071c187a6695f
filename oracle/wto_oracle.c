/*
 * Oracle for the adaptive WENO-theta finite-difference scheme.
 *
 * TEST INFRASTRUCTURE ONLY: a plain FP64 CPU implementation that the tests,
 * the smoke entry point and the benchmark's CPU-baseline leg compare the GPU
 * library against.  The product library shares no source with this file.
 *
 * The code follows the paper step by step, in the paper's order and notation:
 *   Sec. 2        conservative semi-discretisation  L(u)_j = -(F_{j+1/2} - F_{j-1/2})/dx
 *   Sec. 2.1      3rd-order TVD Runge-Kutta
 *   Sec. 2.2      candidate fluxes of S0, S1, S2;  Sec. 2.3 the fourth one of S3
 *   Remark (flux splitting) in Sec. 2.2.2: global Lax-Friedrichs f+- = (f +- alpha u)/2,
 *                 the negative part reconstructed on the mirrored stencil
 *   Sec. 3        linear weights gamma^theta and nonlinear weights omega^theta
 *   Sec. 3.1      central indicators beta~_k, the restriction against alpha_R,
 *                 large-stencil indicators tau_5 and tau_6 and the theta switch;
 *                 epsilon = 1e-10 (remark iii of Sec. 3.1)
 *   Sec. 4.2/4.3  Euler equations, characteristic-wise reconstruction with the
 *                 Roe mean matrix, dimension by dimension in 2D/3D.
 *   Sec. 4.3      TEST 9's boundaries as sides made of two parts (a given
 *                 state, a wall, zero gradient) split at a point that may move;
 *                 wto_step's stages take moving splits at t, t + dt, t + dt/2
 *                 (a reading, pinned by the Simpson-rule error of an inflow
 *                 switched on inside a step).
 *
 * Built with -O2 -ffp-contract=off and without -ffast-math: every operation
 * below is one IEEE double rounding, evaluated left to right as written.
 * Readings where the paper is silent are marked "Reading:".
 */
#include "wto_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define MAXM 5

/* ------------------------------------------------------------------------ */
/* WENO-theta reconstruction of one interface value (Sec. 2.2, 2.3, 3, 3.1) */
/* ------------------------------------------------------------------------ */

/* s[0..5] = f_{j-2}, f_{j-1}, f_j, f_{j+1}, f_{j+2}, f_{j+3}; the value
 * approximates h at x_{j+1/2}. */
static double weno_theta_core(const double s[6], double eps, double alpha_R,
                              double *diag)
{
    const double a = s[0], b = s[1], c = s[2], d = s[3], e = s[4], f = s[5];

    /* Candidate fluxes of S0, S1, S2 (Sec. 2.2) and S3 (Sec. 2.3). */
    const double q0 = (2.0 / 6.0) * a - (7.0 / 6.0) * b + (11.0 / 6.0) * c;
    const double q1 = -(1.0 / 6.0) * b + (5.0 / 6.0) * c + (2.0 / 6.0) * d;
    const double q2 = (2.0 / 6.0) * c + (5.0 / 6.0) * d - (1.0 / 6.0) * e;
    const double q3 = (11.0 / 6.0) * d - (7.0 / 6.0) * e + (2.0 / 6.0) * f;

    /* Central smoothness indicators beta~_0..beta~_3 (Sec. 3.1; beta~_3 on the
     * extended sub-stencil {x_j..x_{j+3}}, in its modified form). */
    double t1, t2;
    t1 = a - 2.0 * b + c;
    t2 = a - 3.0 * b + 2.0 * c;
    double b0 = (13.0 / 12.0) * (t1 * t1) + t2 * t2;
    t1 = b - 2.0 * c + d;
    t2 = d - c;
    double b1 = (13.0 / 12.0) * (t1 * t1) + t2 * t2;
    t1 = c - 2.0 * d + e;
    t2 = c - d;
    double b2 = (13.0 / 12.0) * (t1 * t1) + t2 * t2;
    t1 = 3.0 * c - 7.0 * d + 5.0 * e - f;
    t2 = 2.0 * d - 3.0 * e + f;
    double b3 = (13.0 / 48.0) * (t1 * t1) + t2 * t2;

    if (diag) {
        diag[0] = q0; diag[1] = q1; diag[2] = q2; diag[3] = q3;
        diag[4] = b0; diag[5] = b1; diag[6] = b2; diag[7] = b3;
    }

    /* Restriction (Sec. 3.1): R = max_k beta~_k / (eps + min_k beta~_k);
     * all beta~_k are set to zero when R <= alpha_R. */
    double bmax = b0, bmin = b0;
    if (b1 > bmax) bmax = b1;
    if (b2 > bmax) bmax = b2;
    if (b3 > bmax) bmax = b3;
    if (b1 < bmin) bmin = b1;
    if (b2 < bmin) bmin = b2;
    if (b3 < bmin) bmin = b3;
    const double R = bmax / (eps + bmin);
    int restricted = 0;
    if (R <= alpha_R) {
        b0 = 0.0; b1 = 0.0; b2 = 0.0; b3 = 0.0;
        restricted = 1;
    }

    /* Large-stencil indicators tau_5 (on S^5) and tau_6 (on S^6), Sec. 3.1. */
    t1 = a - 4.0 * b + 6.0 * c - 4.0 * d + e;
    t2 = -b + 3.0 * c - 3.0 * d + e;
    const double tau5 = (13.0 / 12.0) * (t1 * t1) + t2 * t2;
    t1 = -a + 5.0 * b - 10.0 * c + 10.0 * d - 5.0 * e + f;
    t2 = a - 3.0 * b + 2.0 * c + 2.0 * d - 3.0 * e + f;
    const double tau6 = (13.0 / 12.0) * (t1 * t1) + 0.25 * (t2 * t2);

    /* The theta switch: (tau, theta) = (tau6, 0) if tau6 < tau5, else (tau5, 1). */
    double tau, theta;
    if (tau6 < tau5) { tau = tau6; theta = 0.0; }
    else             { tau = tau5; theta = 1.0; }

    /* Linear weights gamma^theta (Sec. 3): theta = 1 gives the 5th-order
     * upwind weights, theta = 0 the 6th-order central ones. */
    const double g0 = (1.0 / 20.0) * (1.0 + theta);
    const double g1 = (3.0 / 20.0) * (3.0 + theta);
    const double g2 = (3.0 / 20.0) * (3.0 - theta);
    const double g3 = (1.0 / 20.0) * (1.0 - theta);

    /* Nonlinear weights omega^theta_k = alpha_k / sum_l alpha_l with
     * alpha_k = gamma_k (1 + tau / (eps + beta~_k)) (Sec. 3). */
    const double al0 = g0 * (1.0 + tau / (eps + b0));
    const double al1 = g1 * (1.0 + tau / (eps + b1));
    const double al2 = g2 * (1.0 + tau / (eps + b2));
    const double al3 = g3 * (1.0 + tau / (eps + b3));
    const double sum = al0 + al1 + al2 + al3;
    const double w0 = al0 / sum, w1 = al1 / sum, w2 = al2 / sum, w3 = al3 / sum;
    const double h = w0 * q0 + w1 * q1 + w2 * q2 + w3 * q3;

    if (diag) {
        diag[8] = R; diag[9] = (double)restricted;
        diag[10] = tau5; diag[11] = tau6; diag[12] = theta;
        diag[13] = w0; diag[14] = w1; diag[15] = w2; diag[16] = w3;
        diag[17] = h; diag[18] = tau;
    }
    return h;
}

double wto_weno_theta(const double s[6], double eps, double alpha_R)
{
    return weno_theta_core(s, eps, alpha_R, NULL);
}

void wto_weno_theta_diag(const double s[6], double eps, double alpha_R,
                         double out[WTO_DIAG_LEN])
{
    weno_theta_core(s, eps, alpha_R, out);
}

/* ------------------------------------------------------------------------ */
/* Grid helpers                                                             */
/* ------------------------------------------------------------------------ */

static int64_t total_points(const wto_problem *P)
{
    return P->n[0] * P->n[1] * P->n[2];
}

static int ncomp(const wto_problem *P)
{
    return P->system == WTO_EULER ? P->ndim + 2 : 1;
}

/* Boundary conditions as index maps onto interior points.  Periodic: wrap.
 * Transmissive (zero gradient): copy the nearest interior point.  Reflective
 * (a wall at the grid's end, half a spacing beyond the outermost point): the
 * mirror image of the point across the wall, whose momentum normal to the wall
 * is negated (see reflected()).
 * Reading: the paper names the conditions (Sec. 3.2, 4.2, 4.3) without giving
 * a ghost-point rule; three ghost points per side are what S^6 needs. */
static int64_t map_index(int64_t i, int64_t n, int32_t bc)
{
    if (bc == WTO_PERIODIC) {
        i %= n;
        if (i < 0) i += n;
        return i;
    }
    if (bc == WTO_REFLECTIVE) {
        if (i < 0) return -1 - i;
        if (i >= n) return 2 * n - 1 - i;
        return i;
    }
    if (i < 0) return 0;
    if (i >= n) return n - 1;
    return i;
}

/* Whether point i of a line of n points is a reflected ghost point. */
static int reflected(int64_t i, int64_t n, int32_t bc)
{
    return bc == WTO_REFLECTIVE && (i < 0 || i >= n);
}

static int64_t stride_of(const wto_problem *P, int d);

/* Part (0 or 1) of side S of dimension d that the ghost points of the grid
 * line starting at offset `base` belong to: 0 where the line's coordinate
 * along the next axis lies below the split point at time P->t.
 * Reading: Sec. 4.3 (TEST 9) gives the bottom and top boundaries as intervals
 * of x on which a rule holds; a ghost point takes the rule of the interval
 * that holds its own line's coordinate, x_j = lo + (j + 1/2) dx, with all
 * three ghost points of a line on the same side of the split. */
static int side_part(const wto_problem *P, int d, int64_t base, const wto_side *S)
{
    if (P->ndim == 1) return 0;
    const int a = (d + 1) % P->ndim;
    const int64_t j = (base / stride_of(P, a)) % P->n[a];
    const double x = P->lo[a] + ((double)j + 0.5) * P->dx[a];
    return x < S->split0 + S->split_speed * P->t ? 0 : 1;
}

/* Conserved state (canonical order) of point i of the grid line along d
 * starting at offset `base`; i may be a ghost point (-3..-1, n..n+2). */
static void line_point(const wto_problem *P, const double *u, int d, int64_t base,
                       int64_t i, double *uc)
{
    const int m = P->ndim + 2;
    const int64_t n = P->n[d], N = P->n[0] * P->n[1] * P->n[2];
    int32_t rule = P->bc[d];
    if (rule == WTO_SIDES) {
        if (i >= 0 && i < n) {
            rule = WTO_TRANSMISSIVE;           /* an interior point: itself */
        } else {
            const wto_side *S = &P->sides[2 * d + (i < 0 ? 0 : 1)];
            const int part = side_part(P, d, base, S);
            rule = S->kind[part];
            if (rule == WTO_STATE) {
                for (int c = 0; c < m; ++c) uc[c] = S->state[part][c];
                return;
            }
        }
    }
    const int64_t cell = base + map_index(i, n, rule) * stride_of(P, d);
    for (int c = 0; c < m; ++c) uc[c] = u[c * N + cell];
    if (reflected(i, n, rule)) uc[1 + d] = -uc[1 + d];
}

static int64_t stride_of(const wto_problem *P, int d)
{
    return d == 0 ? 1 : (d == 1 ? P->n[0] : P->n[0] * P->n[1]);
}

/* Base offset of pencil number p along direction d. */
static int64_t pencil_base(const wto_problem *P, int d, int64_t p)
{
    int o1 = d == 0 ? 1 : 0;
    int o2 = d == 2 ? 1 : 2;
    int64_t i1 = p % P->n[o1];
    int64_t i2 = p / P->n[o1];
    return i1 * stride_of(P, o1) + i2 * stride_of(P, o2);
}

static int validate(const wto_problem *P)
{
    if (!P) return WTO_ERR_ARG;
    if (P->ndim < 1 || P->ndim > 3) return WTO_ERR_ARG;
    if (P->system < WTO_LINEAR || P->system > WTO_EULER) return WTO_ERR_ARG;
    if (P->system != WTO_EULER && P->ndim != 1) return WTO_ERR_UNSUPPORTED;
    for (int d = 0; d < 3; ++d) {
        if (d < P->ndim) {
            if (P->n[d] < 6) return WTO_ERR_ARG;
            if (!(P->dx[d] > 0.0)) return WTO_ERR_ARG;
            if (P->bc[d] != WTO_PERIODIC && P->bc[d] != WTO_TRANSMISSIVE &&
                P->bc[d] != WTO_REFLECTIVE && P->bc[d] != WTO_SIDES)
                return WTO_ERR_ARG;
            if ((P->bc[d] == WTO_REFLECTIVE || P->bc[d] == WTO_SIDES) && P->system != WTO_EULER)
                return WTO_ERR_UNSUPPORTED;
            if (P->bc[d] == WTO_SIDES) {
                if (!P->sides || !isfinite(P->t) || !isfinite(P->lo[(d + 1) % P->ndim]))
                    return WTO_ERR_ARG;
                for (int e = 0; e < 2; ++e) {
                    const wto_side *S = &P->sides[2 * d + e];
                    if (S->split0 != S->split0 || !isfinite(S->split_speed)) return WTO_ERR_ARG;
                    for (int k = 0; k < 2; ++k) {
                        if (S->kind[k] != WTO_TRANSMISSIVE && S->kind[k] != WTO_REFLECTIVE &&
                            S->kind[k] != WTO_STATE)
                            return WTO_ERR_ARG;
                        if (S->kind[k] == WTO_STATE)
                            for (int c = 0; c < P->ndim + 2; ++c)
                                if (!isfinite(S->state[k][c])) return WTO_ERR_ARG;
                    }
                }
            }
        } else if (P->n[d] != 1) {
            return WTO_ERR_ARG;
        }
    }
    if (!(P->eps > 0.0) || !(P->cfl > 0.0)) return WTO_ERR_ARG;
    if (P->alpha_R < 0.0 || P->alpha_R != P->alpha_R) return WTO_ERR_ARG;
    if (P->system == WTO_EULER && !(P->gamma > 1.0)) return WTO_ERR_ARG;
    for (int d = 0; d < 3; ++d) {
        if (!isfinite(P->gravity[d])) return WTO_ERR_ARG;
        if (P->gravity[d] != 0.0 && (P->system != WTO_EULER || d >= P->ndim))
            return WTO_ERR_ARG;
    }
    return WTO_OK;
}

/* ------------------------------------------------------------------------ */
/* Euler equations (Sec. 4.2, 4.3)                                          */
/* ------------------------------------------------------------------------ */

typedef struct {
    double rho, vel[3], E, p, c, H;
} prim_t;

/* Primitive variables of a conserved state in canonical order
 * (rho, m_x, .., E).  Equation of state p = (gamma-1)(E - rho|v|^2/2).
 * Reading: the 2D equation of state in Sec. 4.3 is printed without rho; the
 * 1D form of Sec. 4.2 extended to |v|^2 is used.  The kinetic term sums the
 * velocity components in the order x, y, z. */
static int primitives(const double *uc, int ndim, double gamma, prim_t *P)
{
    const double rho = uc[0];
    const double E = uc[ndim + 1];
    double v2 = 0.0;
    for (int k = 0; k < ndim; ++k) {
        P->vel[k] = uc[1 + k] / rho;
    }
    v2 = P->vel[0] * P->vel[0];
    for (int k = 1; k < ndim; ++k) v2 = v2 + P->vel[k] * P->vel[k];
    const double p = (gamma - 1.0) * (E - 0.5 * rho * v2);
    P->rho = rho;
    P->E = E;
    P->p = p;
    P->c = sqrt(gamma * p / rho);
    P->H = (E + p) / rho;
    if (!(rho == rho) || !(E == E) || !(p == p) || isinf(rho) || isinf(E) || isinf(p))
        return WTO_ERR_NONFINITE;
    if (!(rho > 0.0) || !(p > 0.0)) return WTO_ERR_NONPHYSICAL;
    return WTO_OK;
}

/* Permutation of components for direction d: (rho, m_d, m_t1, m_t2, E),
 * tangential components in increasing axis order.  perm[k] is the canonical
 * index of permuted component k.  All directions then use one routine. */
static void direction_perm(int ndim, int d, int *perm)
{
    perm[0] = 0;
    perm[1] = 1 + d;
    int k = 2;
    for (int e = 0; e < ndim; ++e)
        if (e != d) perm[k++] = 1 + e;
    perm[ndim + 1] = ndim + 1;
}

/* Roe mean state between two cells and the left/right eigenvectors of the
 * Roe matrix in the permuted component order (Sec. 4.2).
 * Reading: the paper cites Roe's mean matrix without formulas; the textbook
 * sqrt(rho)-weighted average of velocity and total enthalpy is used, and
 * the eigenvectors are normalised as below (fixed for parity).
 * Field order: u_n - c, u_n, u_n + c, then one shear field per tangential
 * direction. */
static int roe_eigen(int ndim, int d, double gamma, const prim_t *PL,
                     const prim_t *PR, double L[MAXM][MAXM],
                     double R[MAXM][MAXM], double lam[MAXM])
{
    const int m = ndim + 2;
    const double sl = sqrt(PL->rho);
    const double sr = sqrt(PR->rho);
    const double den = sl + sr;
    double vt[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < ndim; ++k)
        vt[k] = (sl * PL->vel[k] + sr * PR->vel[k]) / den;
    const double H = (sl * PL->H + sr * PR->H) / den;
    double v2 = vt[0] * vt[0];
    for (int k = 1; k < ndim; ++k) v2 = v2 + vt[k] * vt[k];
    const double q2 = 0.5 * v2;
    const double c2 = (gamma - 1.0) * (H - q2);
    if (!(c2 == c2)) return WTO_ERR_NONFINITE;
    if (!(c2 > 0.0)) return WTO_ERR_NONPHYSICAL;
    const double c = sqrt(c2);

    /* normal and tangential velocities in permuted order */
    const double un = vt[d];
    double ut[2] = {0.0, 0.0};
    int nt = 0;
    for (int k = 0; k < ndim; ++k)
        if (k != d) ut[nt++] = vt[k];

    const double b1 = (gamma - 1.0) / c2;
    const double b2 = b1 * q2;
    const double uc = un / c;
    const double ic = 1.0 / c;

    for (int i = 0; i < MAXM; ++i)
        for (int j = 0; j < MAXM; ++j) { L[i][j] = 0.0; R[i][j] = 0.0; }

    /* left eigenvectors (rows) */
    L[0][0] = 0.5 * (b2 + uc);
    L[0][1] = -0.5 * (b1 * un + ic);
    L[1][0] = 1.0 - b2;
    L[1][1] = b1 * un;
    L[2][0] = 0.5 * (b2 - uc);
    L[2][1] = -0.5 * (b1 * un - ic);
    for (int t = 0; t < nt; ++t) {
        L[0][2 + t] = -0.5 * (b1 * ut[t]);
        L[1][2 + t] = b1 * ut[t];
        L[2][2 + t] = -0.5 * (b1 * ut[t]);
        L[3 + t][0] = -ut[t];
        L[3 + t][2 + t] = 1.0;
    }
    L[0][m - 1] = 0.5 * b1;
    L[1][m - 1] = -b1;
    L[2][m - 1] = 0.5 * b1;

    /* right eigenvectors (columns) */
    R[0][0] = 1.0;           R[0][1] = 1.0;  R[0][2] = 1.0;
    R[1][0] = un - c;        R[1][1] = un;   R[1][2] = un + c;
    R[m - 1][0] = H - un * c;
    R[m - 1][1] = q2;
    R[m - 1][2] = H + un * c;
    for (int t = 0; t < nt; ++t) {
        R[2 + t][0] = ut[t];
        R[2 + t][1] = ut[t];
        R[2 + t][2] = ut[t];
        R[2 + t][3 + t] = 1.0;
        R[m - 1][3 + t] = ut[t];
    }

    lam[0] = un - c;
    lam[1] = un;
    lam[2] = un + c;
    for (int t = 0; t < nt; ++t) lam[3 + t] = un;
    return WTO_OK;
}

int wto_euler_eigen(int32_t ndim, int32_t dir, double gamma, const double *uL,
                    const double *uR, double *Lmat, double *Rmat, double *lam)
{
    if (ndim < 1 || ndim > 3 || dir < 0 || dir >= ndim) return WTO_ERR_ARG;
    prim_t PL, PR;
    int st = primitives(uL, ndim, gamma, &PL);
    if (st) return st;
    st = primitives(uR, ndim, gamma, &PR);
    if (st) return st;
    double L[MAXM][MAXM], R[MAXM][MAXM], l[MAXM];
    st = roe_eigen(ndim, dir, gamma, &PL, &PR, L, R, l);
    if (st) return st;
    const int m = ndim + 2;
    for (int i = 0; i < m; ++i) {
        lam[i] = l[i];
        for (int j = 0; j < m; ++j) {
            Lmat[i * m + j] = L[i][j];
            Rmat[i * m + j] = R[i][j];
        }
    }
    return WTO_OK;
}

/* Normal flux of a cell in permuted component order:
 * (m_n, m_n u_n + p, m_n u_t.., u_n (E + p)). */
static void euler_flux_perm(const double *up, const prim_t *P, int ndim, int d,
                            double *fl)
{
    const int m = ndim + 2;
    const double mn = up[1];
    const double un = P->vel[d];
    fl[0] = mn;
    fl[1] = mn * un + P->p;
    int t = 0;
    for (int k = 0; k < ndim; ++k)
        if (k != d) { fl[2 + t] = mn * P->vel[k]; ++t; }
    fl[m - 1] = un * (P->E + P->p);
}

/* Split characteristic stencils at the interface between points i and i+1
 * of the pencil at base along direction d (Sec. 4.2): project the six
 * stencil points onto the characteristic fields of the Roe matrix and split
 * each field with its global Lax-Friedrichs speed.  vp[s] holds the + part on
 * (j-2..j+3); vm[s] holds the - part already mirrored to (j+3..j-2), so that
 * both are reconstructed by the same routine.  R and perm are returned for
 * the back-projection. */
static int euler_interface_stencils(const wto_problem *P, const double *u, int d,
                                    int64_t base, int64_t i, const double *alpha_d,
                                    double vp[MAXM][6], double vm[MAXM][6],
                                    double R[MAXM][MAXM], int *perm)
{
    const int ndim = P->ndim, m = ndim + 2;
    direction_perm(ndim, d, perm);

    double Up[6][MAXM], Fp[6][MAXM];
    prim_t Pk[6];
    for (int k = 0; k < 6; ++k) {
        double uc[MAXM];
        line_point(P, u, d, base, i - 2 + k, uc);
        int st = primitives(uc, ndim, P->gamma, &Pk[k]);
        if (st) return st;
        for (int c = 0; c < m; ++c) Up[k][c] = uc[perm[c]];
        euler_flux_perm(Up[k], &Pk[k], ndim, d, Fp[k]);
    }

    double L[MAXM][MAXM], lam[MAXM];
    int st = roe_eigen(ndim, d, P->gamma, &Pk[2], &Pk[3], L, R, lam);
    if (st) return st;

    /* characteristic projection q = L u, w = L f at each stencil point, then
     * the split v+- = (w +- alpha_s q) / 2 */
    for (int k = 0; k < 6; ++k)
        for (int s = 0; s < m; ++s) {
            double aq = L[s][0] * Up[k][0];
            double aw = L[s][0] * Fp[k][0];
            for (int c = 1; c < m; ++c) {
                aq = aq + L[s][c] * Up[k][c];
                aw = aw + L[s][c] * Fp[k][c];
            }
            vp[s][k] = 0.5 * (aw + alpha_d[s] * aq);
            vm[s][5 - k] = 0.5 * (aw - alpha_d[s] * aq);
        }
    return WTO_OK;
}

/* Numerical flux at that interface: WENO-theta on both split parts of every
 * field, added, then projected back with R.  F is in canonical order. */
static int euler_interface_flux(const wto_problem *P, const double *u, int d,
                                int64_t base, int64_t i, const double *alpha_d,
                                double *F)
{
    const int m = P->ndim + 2;
    double vp[MAXM][6], vm[MAXM][6], R[MAXM][MAXM];
    int perm[MAXM];
    int st = euler_interface_stencils(P, u, d, base, i, alpha_d, vp, vm, R, perm);
    if (st) return st;
    double hs[MAXM];
    for (int s = 0; s < m; ++s)
        hs[s] = weno_theta_core(vp[s], P->eps, P->alpha_R, NULL) +
                weno_theta_core(vm[s], P->eps, P->alpha_R, NULL);

    /* back-projection F = R h.  Reading: the sum over fields takes the two
     * acoustic fields first, then the entropy field, then the shear fields,
     * so that a mirrored state yields exactly the mirrored flux. */
    for (int c = 0; c < m; ++c) {
        double acc = R[c][0] * hs[0] + R[c][2] * hs[2];
        acc = acc + R[c][1] * hs[1];
        for (int s = 3; s < m; ++s) acc = acc + R[c][s] * hs[s];
        F[perm[c]] = acc;
    }
    return WTO_OK;
}

/* Scalar numerical flux at the interface between points i and i+1 of a 1D
 * grid: global LF split of the flux values and WENO-theta on both parts. */
static double scalar_interface_flux(const wto_problem *P, const double *u,
                                    const double *f, double alpha, int64_t i)
{
    double vp[6], vm[6];
    for (int k = 0; k < 6; ++k) {
        const int64_t cell = map_index(i - 2 + k, P->n[0], P->bc[0]);
        vp[k] = 0.5 * (f[cell] + alpha * u[cell]);
        vm[5 - k] = 0.5 * (f[cell] - alpha * u[cell]);
    }
    return weno_theta_core(vp, P->eps, P->alpha_R, NULL) +
           weno_theta_core(vm, P->eps, P->alpha_R, NULL);
}

/* Flux point values of the built-in scalar systems. */
static double scalar_flux(const wto_problem *P, double u)
{
    if (P->system == WTO_LINEAR) return P->a * u;
    return 0.5 * u * u;                    /* Burgers: f(u) = u^2/2 */
}

/* ------------------------------------------------------------------------ */
/* Global LF speeds and the CFL time step                                   */
/* ------------------------------------------------------------------------ */

/* Reading: alpha = max |f'(u)| over the whole domain (Remark on flux
 * splitting) is taken per characteristic field, alpha_s = max |lambda_s|,
 * and re-evaluated from the state of every Runge-Kutta stage.  These are
 * the maxima over the grid's points; pair_wall_speeds() below completes
 * them for reflective walls where the split uses them. */
int wto_alpha(const wto_problem *P, const double *u, double *alpha, double *amax)
{
    int st = validate(P);
    if (st) return st;
    const int ndim = P->ndim, m = ncomp(P);
    const int64_t N = total_points(P);
    if (P->system != WTO_EULER) {
        double am = 0.0;
        for (int64_t j = 0; j < N; ++j) {
            double sp;
            if (!(u[j] == u[j]) || isinf(u[j])) return WTO_ERR_NONFINITE;
            if (P->system == WTO_LINEAR) sp = fabs(P->a);
            else sp = fabs(u[j]);              /* f'(u) = u for Burgers */
            if (sp > am) am = sp;
        }
        alpha[0] = am;
        if (amax) amax[0] = am;
        return WTO_OK;
    }
    for (int k = 0; k < ndim * m; ++k) alpha[k] = 0.0;
    for (int k = 0; k < ndim; ++k) if (amax) amax[k] = 0.0;
    for (int64_t j = 0; j < N; ++j) {
        double uc[MAXM];
        prim_t Pj;
        for (int c = 0; c < m; ++c) uc[c] = u[c * N + j];
        st = primitives(uc, ndim, P->gamma, &Pj);
        if (st) return st;
        for (int d = 0; d < ndim; ++d) {
            const double un = Pj.vel[d];
            double l[MAXM];
            l[0] = fabs(un - Pj.c);
            l[1] = fabs(un);
            l[2] = fabs(un + Pj.c);
            for (int s = 3; s < m; ++s) l[s] = fabs(un);
            for (int s = 0; s < m; ++s)
                if (l[s] > alpha[d * m + s]) alpha[d * m + s] = l[s];
            const double sp = fabs(un) + Pj.c;
            if (amax && sp > amax[d]) amax[d] = sp;
        }
    }
    return WTO_OK;
}

/* Whether dimension d has a wall: reflective ends, or a side with a
 * reflective part. */
static int has_wall(const wto_problem *P, int d)
{
    if (P->bc[d] == WTO_REFLECTIVE) return 1;
    if (P->bc[d] != WTO_SIDES) return 0;
    for (int e = 0; e < 2; ++e)
        for (int k = 0; k < 2; ++k)
            if (P->sides[2 * d + e].kind[k] == WTO_REFLECTIVE) return 1;
    return 0;
}

/* Behind reflective walls in direction d the domain is the mirror-extended
 * one (the ghost points are its point values), where u_d changes sign and
 * the two acoustic fields (u_d - c, u_d + c) exchange their speeds, so over
 * that whole domain both have the larger maximum.  Applied to the speeds the
 * split uses, computed or given, also where only part of a side is a wall. */
static void pair_wall_speeds(const wto_problem *P, double *alpha)
{
    if (P->system != WTO_EULER) return;
    const int m = ncomp(P);
    for (int d = 0; d < P->ndim; ++d)
        if (has_wall(P, d)) {
            double *a = &alpha[d * m];
            const double both = a[2] > a[0] ? a[2] : a[0];
            a[0] = both;
            a[2] = both;
        }
}

/* Reading of "a proper CFL condition" (Sec. 2.1):
 * dt = CFL / sum_d (amax_d / dx_d). */
static double cfl_dt(const wto_problem *P, const double *amax)
{
    double s = amax[0] / P->dx[0];
    for (int d = 1; d < P->ndim; ++d) s = s + amax[d] / P->dx[d];
    return P->cfl / s;
}

/* ------------------------------------------------------------------------ */
/* Spatial operator                                                         */
/* ------------------------------------------------------------------------ */

static int has_gravity(const wto_problem *P)
{
    return P->gravity[0] != 0.0 || P->gravity[1] != 0.0 || P->gravity[2] != 0.0;
}

/* Gravity source (Sec. 4.3, TEST 6: the y-momentum and energy equations gain
 * -g rho and -g rho v).  For an acceleration -g_d along each axis: momentum d
 * gains -(g_d rho) and the energy -(g_x m_x + g_y m_y + g_z m_z), summed in
 * axis order; added to L(u) at point j after the flux divergence. */
static void add_gravity(const wto_problem *P, const double *u, int64_t N, int64_t j,
                        double *Lc, int64_t stride)
{
    const int ndim = P->ndim;
    const double rho = u[j];
    double e = 0.0;
    for (int d = 0; d < ndim; ++d) {
        const double md = u[(1 + d) * N + j];
        Lc[(1 + d) * stride] = Lc[(1 + d) * stride] + (-(P->gravity[d] * rho));
        e = d == 0 ? P->gravity[0] * md : e + P->gravity[d] * md;
    }
    Lc[(ndim + 1) * stride] = Lc[(ndim + 1) * stride] + (-e);
}

int wto_rhs(const wto_problem *P, const double *u, const double *f,
            const double *alpha_in, double *L)
{
    int st = validate(P);
    if (st) return st;
    if (!u || !L) return WTO_ERR_ARG;
    if (f && (P->ndim != 1 || P->system == WTO_EULER)) return WTO_ERR_ARG;
    const int ndim = P->ndim, m = ncomp(P);
    const int64_t N = total_points(P);

    double alpha[3 * MAXM], amax[3];
    if (alpha_in) {
        for (int k = 0; k < ndim * m; ++k) alpha[k] = alpha_in[k];
    } else {
        if (f) return WTO_ERR_ARG;       /* caller-given flux needs its alpha */
        st = wto_alpha(P, u, alpha, amax);
        if (st) return st;
    }
    pair_wall_speeds(P, alpha);

    if (P->system != WTO_EULER) {
        const int64_t n = P->n[0];
        double *fv = (double *)malloc(sizeof(double) * n);
        double *Fh = (double *)malloc(sizeof(double) * (n + 1));
        if (!fv || !Fh) { free(fv); free(Fh); return WTO_ERR_ARG; }
        for (int64_t j = 0; j < n; ++j) fv[j] = f ? f[j] : scalar_flux(P, u[j]);
        /* Fh[j + 1] is the flux at x_{j+1/2}, j = -1..n-1 */
        for (int64_t j = -1; j < n; ++j)
            Fh[j + 1] = scalar_interface_flux(P, u, fv, alpha[0], j);
        /* L(u)_j = -(F_{j+1/2} - F_{j-1/2}) / dx */
        for (int64_t j = 0; j < n; ++j)
            L[j] = -((Fh[j + 1] - Fh[j]) / P->dx[0]);
        free(fv);
        free(Fh);
        return WTO_OK;
    }

    /* Euler: dimension by dimension.  D_d = (F_{i+1/2} - F_{i-1/2}) / dx_d
     * per direction; L = -(D_x + D_y + D_z), summed in direction order. */
    double *D = (double *)calloc((size_t)(m * N), sizeof(double));
    if (!D) return WTO_ERR_ARG;
    int err = WTO_OK;
    for (int d = 0; d < ndim; ++d) {
        const int64_t nd = P->n[d];
        const int64_t npen = N / nd;
        const int64_t sd = stride_of(P, d);
        #pragma omp parallel for schedule(static)
        for (int64_t pn = 0; pn < npen; ++pn) {
            const int64_t base = pencil_base(P, d, pn);
            double *Fh = (double *)malloc(sizeof(double) * (size_t)((nd + 1) * m));
            int lerr = Fh ? WTO_OK : WTO_ERR_ARG;
            for (int64_t i = -1; i < nd && !lerr; ++i)
                lerr = euler_interface_flux(P, u, d, base, i, &alpha[d * m],
                                            &Fh[(i + 1) * m]);
            if (!lerr) {
                for (int64_t i = 0; i < nd; ++i)
                    for (int c = 0; c < m; ++c) {
                        const double Dd = (Fh[(i + 1) * m + c] - Fh[i * m + c]) / P->dx[d];
                        const int64_t idx = c * N + base + i * sd;
                        D[idx] = d == 0 ? Dd : D[idx] + Dd;
                    }
            } else {
                #pragma omp critical
                { if (!err) err = lerr; }
            }
            free(Fh);
        }
        if (err) break;
    }
    if (!err) {
        for (int64_t k = 0; k < m * N; ++k) L[k] = -D[k];
        if (has_gravity(P))
            for (int64_t j = 0; j < N; ++j) add_gravity(P, u, N, j, &L[j], N);
    }
    free(D);
    return err;
}

int wto_rhs_points(const wto_problem *P, const double *u, const double *alpha_in,
                   const int64_t *cells, int64_t npts, double *Lpts)
{
    int st = validate(P);
    if (st) return st;
    if (P->system != WTO_EULER && P->ndim != 1) return WTO_ERR_UNSUPPORTED;
    const int ndim = P->ndim, m = ncomp(P);
    const int64_t N = total_points(P);
    double alpha[3 * MAXM], amax[3];
    if (alpha_in) {
        for (int k = 0; k < ndim * m; ++k) alpha[k] = alpha_in[k];
    } else {
        st = wto_alpha(P, u, alpha, amax);
        if (st) return st;
    }
    pair_wall_speeds(P, alpha);
    for (int64_t k = 0; k < npts; ++k) {
        const int64_t cell = cells[k];
        if (cell < 0 || cell >= N) return WTO_ERR_ARG;
        int64_t coord[3] = {cell % P->n[0], (cell / P->n[0]) % P->n[1],
                            cell / (P->n[0] * P->n[1])};
        if (P->system != WTO_EULER) {
            const int64_t n = P->n[0];
            double *fv = (double *)malloc(sizeof(double) * n);
            if (!fv) return WTO_ERR_ARG;
            for (int64_t j = 0; j < n; ++j) fv[j] = scalar_flux(P, u[j]);
            const double Fr = scalar_interface_flux(P, u, fv, alpha[0], coord[0]);
            const double Fl = scalar_interface_flux(P, u, fv, alpha[0], coord[0] - 1);
            free(fv);
            Lpts[k] = -((Fr - Fl) / P->dx[0]);
            continue;
        }
        double Dsum[MAXM];
        for (int d = 0; d < ndim; ++d) {
            const int64_t sd = stride_of(P, d);
            const int64_t base = cell - coord[d] * sd;
            double Fr[MAXM], Fl[MAXM];
            st = euler_interface_flux(P, u, d, base, coord[d], &alpha[d * m], Fr);
            if (st) return st;
            st = euler_interface_flux(P, u, d, base, coord[d] - 1, &alpha[d * m], Fl);
            if (st) return st;
            for (int c = 0; c < m; ++c) {
                const double Dd = (Fr[c] - Fl[c]) / P->dx[d];
                Dsum[c] = d == 0 ? Dd : Dsum[c] + Dd;
            }
        }
        for (int c = 0; c < m; ++c) Lpts[k * m + c] = -Dsum[c];
        if (has_gravity(P)) add_gravity(P, u, N, cell, &Lpts[k * m], 1);
    }
    return WTO_OK;
}

/* ------------------------------------------------------------------------ */
/* Time integration (Sec. 2.1)                                              */
/* ------------------------------------------------------------------------ */

int wto_step(const wto_problem *P, double *u, double dt, double *dt_used)
{
    int st = validate(P);
    if (st) return st;
    const int m = ncomp(P);
    const int64_t M = m * total_points(P);
    double alpha[3 * MAXM], amax[3];
    st = wto_alpha(P, u, alpha, amax);
    if (st) return st;
    if (!(dt > 0.0)) dt = cfl_dt(P, amax);
    if (dt_used) *dt_used = dt;

    double *L = (double *)malloc(sizeof(double) * M);
    double *u1 = (double *)malloc(sizeof(double) * M);
    double *u2 = (double *)malloc(sizeof(double) * M);
    if (!L || !u1 || !u2) { free(L); free(u1); free(u2); return WTO_ERR_ARG; }

    /* Reading: boundary data that move (WTO_SIDES splits) are taken at the
     * times the stages approximate, t^n, t^n + dt and t^n + dt/2 (the
     * abscissae of the 3-stage scheme); the paper states none. */
    wto_problem Q = *P;

    /* u(1) = u^n + dt L(u^n) */
    Q.t = P->t;
    st = wto_rhs(&Q, u, NULL, alpha, L);
    if (!st) {
        for (int64_t k = 0; k < M; ++k) u1[k] = u[k] + dt * L[k];
        /* u(2) = 3/4 u^n + 1/4 u(1) + 1/4 dt L(u(1)) */
        Q.t = P->t + dt;
        st = wto_rhs(&Q, u1, NULL, NULL, L);
    }
    if (!st) {
        for (int64_t k = 0; k < M; ++k)
            u2[k] = 0.75 * u[k] + 0.25 * u1[k] + 0.25 * dt * L[k];
        /* u^{n+1} = 1/3 u^n + 2/3 u(2) + 2/3 dt L(u(2)) */
        Q.t = P->t + 0.5 * dt;
        st = wto_rhs(&Q, u2, NULL, NULL, L);
    }
    if (!st)
        for (int64_t k = 0; k < M; ++k)
            u[k] = (1.0 / 3.0) * u[k] + (2.0 / 3.0) * u2[k] + (2.0 / 3.0) * dt * L[k];
    free(L);
    free(u1);
    free(u2);
    return st;
}

int wto_solve(const wto_problem *P, double *u, double t0, double t_end,
              int64_t max_steps, double *t_out, int64_t *steps_out)
{
    int st = validate(P);
    if (st) return st;
    double t = t0;
    int64_t steps = 0;
    wto_problem Q = *P;
    while (t < t_end && (max_steps < 0 || steps < max_steps)) {
        double alpha[3 * MAXM], amax[3];
        st = wto_alpha(P, u, alpha, amax);
        if (st) break;
        double dt = cfl_dt(P, amax);
        /* Reading: the last step is clipped to end exactly at t_end; a step that
         * would leave less than 1e-6 dt to go is stretched to t_end instead of
         * being followed by a round-off-sized step. */
        int last = 0;
        if (t + dt >= t_end - 1e-6 * dt) { dt = t_end - t; last = 1; }
        Q.t = t;
        st = wto_step(&Q, u, dt, NULL);
        if (st) break;
        t = last ? t_end : t + dt;
        ++steps;
    }
    if (t_out) *t_out = t;
    if (steps_out) *steps_out = steps;
    return st;
}

/* ------------------------------------------------------------------------ */
/* Decisions and their margins, for flip accounting                         */
/* ------------------------------------------------------------------------ */

/* theta (tau_6 < tau_5) and the restriction (R <= alpha_R) are discontinuous in
 * the six stencil values (Sec. 3.1), so an evaluation of the same formulas with
 * other rounding (another operation order, fused multiply-adds) may legitimately
 * take the other branch where the two sides of a comparison are closer than
 * their rounding errors.  decisions_core reports each decision with its margin
 * in units of a first-order bound on those errors: |tau_6 - tau_5| / (E_5 + E_6)
 * and |R - alpha_R| / E_R, where E bounds the error of a quantity computed in
 * double precision from stencil values that themselves carry errors of up to
 * err_s[k] (the projection and split that form them).  A margin below a few
 * units marks a near-tie; +inf marks a comparison no rounding can change (both
 * sides exactly zero, as for a constant stencil). */

#define WTO_U 0x1p-53

/* Error bound of t = sum_i c[i] s[i] (n terms) from the rounding of the sum and
 * the errors err_s of the values. */
static double lin_err(const double *c, const double *s, const double *err_s, int first, int n)
{
    double e = 0.0, mag = 0.0;
    for (int i = 0; i < n; ++i) {
        mag += fabs(c[i] * s[first + i]);
        e += fabs(c[i]) * err_s[first + i];
    }
    return e + (double)(n + 1) * WTO_U * mag;
}

/* Error bound of A t1^2 + B t2^2 with t1, t2 the combinations (c1, c2) of the
 * stencil; value returned in *val. */
static double sq_err(double A, const double *c1, int f1, int n1, double B, const double *c2,
                     int f2, int n2, const double *s, const double *err_s, double *val)
{
    double t1 = 0.0, t2 = 0.0;
    for (int i = 0; i < n1; ++i) t1 += c1[i] * s[f1 + i];
    for (int i = 0; i < n2; ++i) t2 += c2[i] * s[f2 + i];
    *val = A * t1 * t1 + B * t2 * t2;
    return 2.0 * A * fabs(t1) * lin_err(c1, s, err_s, f1, n1) +
           2.0 * B * fabs(t2) * lin_err(c2, s, err_s, f2, n2) + 4.0 * WTO_U * *val;
}

static double scaled_margin(double diff, double err)
{
    if (err > 0.0) return fabs(diff) / err;
    return INFINITY;
}

/* out: theta, restricted (as the reconstruction decides them), theta margin,
 * restriction margin. */
static void decisions_core(const double s[6], const double err_s[6], double eps,
                           double alpha_R, int32_t *theta, int32_t *restricted,
                           double *m_theta, double *m_restr)
{
    double d[WTO_DIAG_LEN];
    weno_theta_core(s, eps, alpha_R, d);
    *theta = (int32_t)d[12];
    *restricted = (int32_t)d[9];

    /* beta~_k and tau (Sec. 3.1) with their error bounds */
    static const double c_b0a[3] = {1.0, -2.0, 1.0}, c_b0b[3] = {1.0, -3.0, 2.0};
    static const double c_b1a[3] = {1.0, -2.0, 1.0}, c_b1b[2] = {-1.0, 1.0};
    static const double c_b2a[3] = {1.0, -2.0, 1.0}, c_b2b[2] = {1.0, -1.0};
    static const double c_b3a[4] = {3.0, -7.0, 5.0, -1.0}, c_b3b[3] = {2.0, -3.0, 1.0};
    static const double c_t5a[5] = {1.0, -4.0, 6.0, -4.0, 1.0}, c_t5b[4] = {-1.0, 3.0, -3.0, 1.0};
    static const double c_t6a[6] = {-1.0, 5.0, -10.0, 10.0, -5.0, 1.0};
    static const double c_t6b[6] = {1.0, -3.0, 2.0, 2.0, -3.0, 1.0};
    double b[4], eb[4], t5, t6;
    eb[0] = sq_err(13.0 / 12.0, c_b0a, 0, 3, 1.0, c_b0b, 0, 3, s, err_s, &b[0]);
    eb[1] = sq_err(13.0 / 12.0, c_b1a, 1, 3, 1.0, c_b1b, 2, 2, s, err_s, &b[1]);
    eb[2] = sq_err(13.0 / 12.0, c_b2a, 2, 3, 1.0, c_b2b, 2, 2, s, err_s, &b[2]);
    eb[3] = sq_err(13.0 / 48.0, c_b3a, 2, 4, 1.0, c_b3b, 3, 3, s, err_s, &b[3]);
    const double e5 = sq_err(13.0 / 12.0, c_t5a, 0, 5, 1.0, c_t5b, 1, 4, s, err_s, &t5);
    const double e6 = sq_err(13.0 / 12.0, c_t6a, 0, 6, 0.25, c_t6b, 0, 6, s, err_s, &t6);
    *m_theta = scaled_margin(d[11] - d[10], e5 + e6);

    int kmax = 0, kmin = 0;
    for (int k = 1; k < 4; ++k) {
        if (b[k] > b[kmax]) kmax = k;
        if (b[k] < b[kmin]) kmin = k;
    }
    const double R = d[8];
    double eR = 0.0;
    if (R > 0.0 && isfinite(R))
        eR = R * ((b[kmax] > 0.0 ? eb[kmax] / b[kmax] : 0.0) + eb[kmin] / (eps + b[kmin]) +
                  2.0 * WTO_U);
    *m_restr = scaled_margin(R - alpha_R, eR);
}

/* Absolute scale of the split values v+-_{s,k} = (w +- alpha_s q)/2 for the
 * error bounds: (sum_c |L_sc f_c| + alpha_s sum_c |L_sc u_c|) / 2 times the
 * roundings of the projection (m products, m - 1 sums) and of the split. */
static void euler_split_errors(const wto_problem *P, const double *u, int d, int64_t base,
                               int64_t i, const double *alpha_d, double ep[MAXM][6],
                               double em[MAXM][6])
{
    const int ndim = P->ndim, m = ndim + 2;
    int perm[MAXM];
    direction_perm(ndim, d, perm);
    double Up[6][MAXM], Fp[6][MAXM];
    prim_t Pk[6];
    for (int k = 0; k < 6; ++k) {
        double uc[MAXM];
        line_point(P, u, d, base, i - 2 + k, uc);
        primitives(uc, ndim, P->gamma, &Pk[k]);
        for (int c = 0; c < m; ++c) Up[k][c] = uc[perm[c]];
        euler_flux_perm(Up[k], &Pk[k], ndim, d, Fp[k]);
    }
    double L[MAXM][MAXM], R[MAXM][MAXM], lam[MAXM];
    roe_eigen(ndim, d, P->gamma, &Pk[2], &Pk[3], L, R, lam);
    for (int k = 0; k < 6; ++k)
        for (int s = 0; s < m; ++s) {
            double sq = 0.0, sw = 0.0;
            for (int c = 0; c < m; ++c) {
                sq += fabs(L[s][c] * Up[k][c]);
                sw += fabs(L[s][c] * Fp[k][c]);
            }
            const double e = (double)(m + 3) * WTO_U * 0.5 * (sw + alpha_d[s] * sq);
            ep[s][k] = e;
            em[s][5 - k] = e;
        }
}

int wto_decisions(const wto_problem *P, const double *u, const double *alpha_in, int32_t dir,
                  int32_t *dec, double *margins)
{
    int st = validate(P);
    if (st) return st;
    if (!u || !dec || !margins) return WTO_ERR_ARG;
    if (dir < 0 || dir >= P->ndim) return WTO_ERR_ARG;
    const int ndim = P->ndim, m = ncomp(P);
    double alpha[3 * MAXM], amax[3];
    if (alpha_in) {
        for (int k = 0; k < ndim * m; ++k) alpha[k] = alpha_in[k];
    } else {
        st = wto_alpha(P, u, alpha, amax);
        if (st) return st;
    }
    pair_wall_speeds(P, alpha);
    const int64_t nd = P->n[dir];
    const int64_t npen = total_points(P) / nd;
    /* output strides: the grid with dimension dir extended to nd + 1 interfaces */
    int64_t ext[3] = {P->n[0], P->n[1], P->n[2]};
    ext[dir] = nd + 1;
    const int64_t es[3] = {1, ext[0], ext[0] * ext[1]};
    for (int64_t pn = 0; pn < npen && !st; ++pn) {
        const int64_t base = pencil_base(P, dir, pn);
        const int64_t coord[3] = {base % P->n[0], (base / P->n[0]) % P->n[1],
                                  base / (P->n[0] * P->n[1])};
        int64_t obase = 0;
        for (int k = 0; k < 3; ++k)
            if (k != dir) obase += coord[k] * es[k];
        for (int64_t i = -1; i < nd && !st; ++i) {
            double vp[MAXM][6], vm[MAXM][6], ep[MAXM][6], em[MAXM][6];
            if (P->system != WTO_EULER) {
                for (int k = 0; k < 6; ++k) {
                    const int64_t cell = map_index(i - 2 + k, nd, P->bc[0]);
                    const double fv = scalar_flux(P, u[cell]);
                    vp[0][k] = 0.5 * (fv + alpha[0] * u[cell]);
                    vm[0][5 - k] = 0.5 * (fv - alpha[0] * u[cell]);
                    const double e = 3.0 * WTO_U * 0.5 * (fabs(fv) + fabs(alpha[0] * u[cell]));
                    ep[0][k] = e;
                    em[0][5 - k] = e;
                }
            } else {
                double R[MAXM][MAXM];
                int perm[MAXM];
                st = euler_interface_stencils(P, u, dir, base, i, &alpha[dir * m], vp, vm, R, perm);
                if (st) break;
                euler_split_errors(P, u, dir, base, i, &alpha[dir * m], ep, em);
            }
            const int64_t o = obase + (i + 1) * es[dir];
            for (int s = 0; s < m; ++s) {
                int32_t *dd = &dec[(o * m + s) * 4];
                double *mm = &margins[(o * m + s) * 4];
                decisions_core(vp[s], ep[s], P->eps, P->alpha_R, &dd[0], &dd[1], &mm[0], &mm[1]);
                decisions_core(vm[s], em[s], P->eps, P->alpha_R, &dd[2], &dd[3], &mm[2], &mm[3]);
            }
        }
    }
    return st;
}
