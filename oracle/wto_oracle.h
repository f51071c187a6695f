/*
 * Oracle for the adaptive WENO-theta finite-difference scheme (Jung & Nguyen,
 * "A New Adaptive WENO-theta Scheme for Hyperbolic Conservation Laws").
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, serial-per-element FP64 CPU
 * implementation used to check the GPU library.  Only the test suite, the
 * smoke entry point and the benchmark's CPU-baseline leg may load it.  The
 * product library shares no source with it and never calls it.
 *
 * All arrays are host arrays.  A state array holds m components of point
 * values, component-major, x fastest: u[c][z][y][x] (no ghost points).
 */
#ifndef WTO_ORACLE_H
#define WTO_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { WTO_OK = 0, WTO_ERR_ARG = 1, WTO_ERR_UNSUPPORTED = 2,
       WTO_ERR_NONPHYSICAL = 3, WTO_ERR_NONFINITE = 4 };
enum { WTO_LINEAR = 0, WTO_BURGERS = 1, WTO_EULER = 2 };
enum { WTO_PERIODIC = 0, WTO_TRANSMISSIVE = 1, WTO_REFLECTIVE = 2, WTO_SIDES = 3 };
/* Rule of one part of a side (bc WTO_SIDES): WTO_TRANSMISSIVE, WTO_REFLECTIVE,
 * or WTO_STATE, a given state in every ghost point. */
enum { WTO_STATE = 3 };

/* One end of one dimension d whose bc is WTO_SIDES (Euler only).  The ghost
 * points beyond that end on the grid line through coordinate x along the next
 * axis a = (d + 1) mod ndim, x = lo[a] + (j + 1/2) dx[a] for the line's index
 * j, follow the rule kind[0] where x < split0 + split_speed * t, else kind[1]
 * (1D: always kind[0]).  A WTO_STATE part puts the conserved state state[part]
 * (rho, m_x, .., E; m entries) into each ghost point.  This describes the
 * boundaries of Sec. 4.3 TEST 9: inflow of a given state, a wall on part of
 * a side and the given state on the rest, and a side whose given state
 * changes at a point that moves with the shock. */
typedef struct {
    int32_t kind[2];
    double  state[2][5];
    double  split0;
    double  split_speed;
} wto_side;

typedef struct {
    int32_t ndim;      /* 1, 2 or 3 (scalar systems: 1 only)                 */
    int32_t system;    /* WTO_LINEAR (f = a u), WTO_BURGERS (f = u^2/2), WTO_EULER */
    int64_t n[3];      /* points per dimension (n[k] = 1 for k >= ndim)     */
    double  dx[3];     /* grid spacing per dimension                        */
    int32_t bc[3];     /* WTO_PERIODIC, WTO_TRANSMISSIVE, WTO_REFLECTIVE or
                          WTO_SIDES (Euler only) per dimension               */
    double  a;         /* advection speed of WTO_LINEAR                     */
    double  gamma;     /* ratio of specific heats (Euler)                   */
    double  cfl;       /* CFL number                                        */
    double  eps;       /* epsilon of the nonlinear weights (1e-10)          */
    double  alpha_R;   /* restriction threshold; 0 disables, +inf = linear  */
    double  gravity[3];/* Euler: gravitational acceleration g_d along -x_d;
                          source (0, -rho g, -(g . m)) (Sec. 4.3, TEST 6)   */
    double  lo[3];     /* coordinate of the domain's lower end per dimension
                          (grid line coordinates of the WTO_SIDES splits)   */
    const wto_side *sides; /* 6 sides [d][lower, upper end], read where
                          bc[d] == WTO_SIDES (NULL if none)                 */
    double  t;         /* time of the state: wto_rhs evaluates moving splits
                          at t; wto_step advances from t (its stages at t,
                          t + dt, t + dt/2); wto_solve ignores it (uses t0)  */
} wto_problem;

/* Number of diagnostic values written by wto_weno_theta_diag. */
#define WTO_DIAG_LEN 19

/* One WENO-theta reconstruction of the interface value from six stencil
 * values s[0..5] = f_{j-2}..f_{j+3}.  Returns the reconstructed value. */
double wto_weno_theta(const double s[6], double eps, double alpha_R);

/* Same, also reporting intermediates:
 * out = {q0,q1,q2,q3, b0,b1,b2,b3 (before restriction), R, restricted,
 *        tau5, tau6, theta, w0,w1,w2,w3, h, tau}. */
void wto_weno_theta_diag(const double s[6], double eps, double alpha_R,
                         double out[WTO_DIAG_LEN]);

/* Roe-averaged eigen-system of the Euler flux in direction dir between the
 * conserved states uL and uR (canonical order rho, m_x.., E).  Lmat and Rmat
 * are m x m row-major in the permuted component order (rho, m_normal,
 * m_tangential.., E); lam[m] are the eigenvalues.  Returns a status. */
int wto_euler_eigen(int32_t ndim, int32_t dir, double gamma, const double *uL,
                    const double *uR, double *Lmat, double *Rmat, double *lam);

/* Global Lax-Friedrichs speeds alpha[d*m + s] = max over all points of
 * |lambda_s| in direction d, and amax[d] = max over all points of the
 * largest wave speed in direction d (|u_d| + c for Euler, |f'(u)| scalar). */
int wto_alpha(const wto_problem *P, const double *u, double *alpha, double *amax);

/* Spatial operator L(u) of the conservative semi-discretisation.
 * f: optional caller-evaluated flux point values (1D scalar only; NULL means
 * the flux of P->system).  alpha: optional LF speeds [ndim*m] (NULL means
 * computed by wto_alpha). */
int wto_rhs(const wto_problem *P, const double *u, const double *f,
            const double *alpha, double *L);

/* L(u) at selected points only (flattened x-fastest indices), written as
 * Lpts[k*m + c].  alpha as in wto_rhs. */
int wto_rhs_points(const wto_problem *P, const double *u, const double *alpha,
                   const int64_t *cells, int64_t npts, double *Lpts);

/* One 3-stage TVD Runge-Kutta step in place.  dt > 0 is used as given,
 * dt <= 0 selects the CFL step.  *dt_used receives the step taken. */
int wto_step(const wto_problem *P, double *u, double dt, double *dt_used);

/* Advance from t0 to t_end with CFL steps (the last one clipped to t_end), or
 * until max_steps steps (max_steps < 0: unlimited). */
int wto_solve(const wto_problem *P, double *u, double t0, double t_end,
              int64_t max_steps, double *t_out, int64_t *steps_out);

/* Decisions of every reconstruction along direction dir, for flip accounting:
 * for each interface (i + 1/2, i = -1..n_dir - 1, of each grid line along dir)
 * and field s, the theta and restriction decisions of the + and - parts and
 * their margins in units of a first-order bound on the rounding errors of the
 * compared quantities (|tau_6 - tau_5| / (E_5 + E_6), |R - alpha_R| / E_R,
 * the stencil values' own errors from the projection and split included;
 * +inf where no rounding can change the comparison).  dec and margins have
 * shape [ext_z][ext_y][ext_x][m][4], ext the grid's point counts with
 * ext_dir = n_dir + 1 (entry i + 1 for interface i + 1/2); the last axis is
 * [theta+, restricted+, theta-, restricted-] and the margins in that order.
 * alpha as in wto_rhs. */
int wto_decisions(const wto_problem *P, const double *u, const double *alpha,
                  int32_t dir, int32_t *dec, double *margins);

#ifdef __cplusplus
}
#endif
#endif
