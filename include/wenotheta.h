/*
 * wenotheta.h -- C ABI of the MI355X (gfx950) WENO-theta library.
 *
 * The library advances hyperbolic conservation laws u_t + f(u)_x (+ g(u)_y
 * + h(u)_z) = 0 with the adaptive WENO-theta finite-difference scheme of
 * Jung & Nguyen ("A New Adaptive WENO-theta Scheme for Hyperbolic
 * Conservation Laws"):
 *   - point values on a uniform grid and the conservative semi-discretisation
 *     L(u)_j = -(F_{j+1/2} - F_{j-1/2}) / dx (Sec. 2);
 *   - global Lax-Friedrichs flux splitting, the negative part reconstructed on
 *     the mirrored stencil (Sec. 2.2.2, remark on flux splitting);
 *   - WENO-theta reconstruction: four 3-point candidate fluxes, central
 *     smoothness indicators beta~_k with the alpha_R restriction, the
 *     large-stencil indicators tau_5 / tau_6 and the theta switch between the
 *     5th-order upwind and 6th-order central linear weights (Sec. 3, 3.1);
 *   - for the Euler equations, characteristic-wise reconstruction with the Roe
 *     mean matrix (Sec. 4.2), dimension by dimension in 2D and 3D (Sec. 4.3);
 *   - 3rd-order TVD Runge-Kutta in time (Sec. 2.1).
 *
 * Conventions for every entry point:
 *   - C symbols only; nothing throws across the ABI; every call returns a
 *     wt_status (WT_OK = 0).
 *   - Array arguments are DEVICE pointers unless stated otherwise.  A state
 *     holds m components of FP64 point values, component-major, x fastest:
 *     u[c][z][y][x], no ghost points.  m = 1 for the scalar systems, ndim + 2
 *     for Euler with components (rho, rho*u_x, [rho*u_y, [rho*u_z,]] E).
 *   - The caller owns u, f and L.  The library owns only the context's
 *     workspace (stage buffers, reduction slots, device scalars), allocated
 *     lazily on the first call with a given size and kept until the context
 *     is destroyed; calls after that allocate nothing.
 *   - Work is ordered on the given stream (a hipStream_t passed as void*;
 *     NULL = the default stream).  Calls on one context must be issued on one
 *     stream and must not overlap.
 *   - Argument errors are detected on the host, before any work is queued,
 *     and returned synchronously.  States the device finds non-physical
 *     (rho <= 0, p <= 0) or non-finite are recorded in the context and
 *     returned by the next synchronising call (wenotheta_sync,
 *     wenotheta_solve); the contents of u are then unspecified.
 */
#ifndef WENOTHETA_H
#define WENOTHETA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    WT_OK = 0,
    WT_ERR_ARG = 1,          /* invalid argument (checked on the host)        */
    WT_ERR_UNSUPPORTED = 2,  /* valid but not provided (e.g. scalar in 2D)    */
    WT_ERR_NONPHYSICAL = 3,  /* rho <= 0 or p <= 0 met on the device          */
    WT_ERR_NONFINITE = 4,    /* NaN or Inf met on the device                  */
    WT_ERR_DEVICE = 5,       /* HIP runtime error                             */
    WT_ERR_NOMEM = 6,        /* workspace allocation failed                   */
    WT_ERR_SCRATCH = 7       /* input exceeds the fixed scratch buffer of
                                wenotheta_rhs_noalloc                         */
} wt_status;

typedef enum {
    WT_LINEAR = 0,   /* f(u) = a u                       (scalar, 1D) */
    WT_BURGERS = 1,  /* f(u) = u^2 / 2                   (scalar, 1D) */
    WT_EULER = 2     /* Euler equations of gas dynamics, 1D/2D/3D      */
} wt_system;

typedef enum {
    WT_PERIODIC = 0,     /* wrap-around                                     */
    WT_TRANSMISSIVE = 1, /* zero gradient: ghost points copy the nearest point */
    WT_REFLECTIVE = 2,   /* wall half a spacing beyond the end points (Euler
                            only; Sec. 4.2 TEST 5, Sec. 4.3 TESTs 6, 7): ghost
                            points are the mirror images of the points across
                            the wall, with the momentum normal to it negated;
                            the split of that direction gives the two acoustic
                            fields (u_d -+ c) the larger of their two maximum
                            speeds, computed or given, as over the mirror-
                            extended domain where they exchange speeds */
    WT_SIDES = 3         /* Euler only: each end follows its entry of the
                            context's side table (wenotheta_set_sides)       */
} wt_bc;

/* Rule of one part of a side. */
typedef enum {
    WT_SIDE_TRANSMISSIVE = 1, /* zero gradient, as WT_TRANSMISSIVE           */
    WT_SIDE_REFLECTIVE = 2,   /* a wall, as WT_REFLECTIVE (a dimension with a
                                 wall part anywhere pairs its acoustic speeds) */
    WT_SIDE_STATE = 3         /* every ghost point holds the given state     */
} wt_side_kind;

/* One end of one dimension d of a grid whose bc[d] is WT_SIDES (Sec. 4.3,
 * TEST 9: inflow of a given state; a wall on part of a side and a given state
 * on the rest; a side whose given state changes at a point moving with a
 * shock).  The ghost points beyond that end on the grid line with coordinate
 * x = lo[a] + (j + 1/2) dx_a along the next axis a = (d + 1) mod ndim follow
 * kind[0] where x < split0 + split_speed * t, kind[1] elsewhere (1D: always
 * kind[0]); t is the time of the state being differentiated.  A
 * WT_SIDE_STATE part puts the conserved state state[part] (rho, m_x, ..., E:
 * ndim + 2 entries) into each of the line's ghost points. */
typedef struct {
    int32_t kind[2];      /* wt_side_kind of part 0 and part 1              */
    double state[2][5];   /* given states of WT_SIDE_STATE parts            */
    double split0;        /* split point at t = 0 (+-inf: one part only)    */
    double split_speed;   /* its speed (finite)                             */
} wt_side;

typedef enum {
    WT_FP64 = 0,         /* every step in IEEE double precision, in the plain
                            order of the formulas (bit-reproducible)          */
    WT_FP32_RECON = 1,   /* the nonlinear weights of the WENO-theta
                            reconstructions (Sec. 3: alpha_k from tau and the
                            beta~_k) in FP32; the candidate fluxes, the
                            indicators, the theta and restriction decisions,
                            the weighted sum, projections, fluxes, RK stages
                            and all stored states stay FP64                  */
    WT_FP64_FAST = 2     /* every step in FP64 with fused multiply-adds and
                            fast (not correctly rounded) reciprocals and
                            square roots; where the restriction holds, the
                            weights are the linear weights gamma^theta exactly
                            (Sec. 3.1).  Differs from WT_FP64 by rounding; a
                            theta or restriction decision may differ where its
                            two sides are within rounding of each other       */
} wt_precision;

/* Uniform grid.  n[k] points in dimension k (n[k] = 1 for k >= ndim; at least
 * 6 for k < ndim), spacing dx_k = (hi[k] - lo[k]) / n[k], boundary condition
 * bc[k] applied at both ends of dimension k. */
typedef struct {
    int32_t ndim;
    int32_t reserved0;
    int64_t n[3];
    double lo[3];
    double hi[3];
    int32_t bc[3];
    int32_t reserved1;
} wt_grid;

/* Scheme parameters. */
typedef struct {
    int32_t system;     /* wt_system                                          */
    int32_t precision;  /* wt_precision                                       */
    double a;           /* advection speed of WT_LINEAR                       */
    double gamma;       /* ratio of specific heats (> 1), Euler (Sec. 4.2: 1.4) */
    double cfl;         /* CFL number (> 0), e.g. 0.5 (Sec. 4.3)              */
    double eps;         /* epsilon of the nonlinear weights (> 0), 1e-10 (Sec. 3.1) */
    double alpha_R;     /* restriction threshold of beta~_k (>= 0; 0 switches it
                           off, +inf gives the linear weights), 50 (Sec. 4.2) */
    double gravity[3];  /* Euler: gravitational acceleration g_d pointing along
                           -x_d (finite; 0 beyond ndim).  The source of Sec. 4.3
                           TEST 6 is added to L: momentum d gains -g_d rho, the
                           energy -(g_x m_x + g_y m_y + g_z m_z).  All 0: none. */
} wt_params;

typedef struct wt_ctx wt_ctx;

/* Create a context bound to HIP device `device`.  *ctx receives the handle. */
wt_status wenotheta_ctx_create(wt_ctx **ctx, int32_t device);

/* Free the context and its workspace (synchronises the device first). */
wt_status wenotheta_ctx_destroy(wt_ctx *ctx);

/* Static description of a status code. */
const char *wenotheta_status_string(int32_t status);

/* Spatial operator L = L(u) of the semi-discretisation (Sec. 2): writes m
 * components of L(u) for every grid point into L_out (device, same layout as
 * u).  The Lax-Friedrichs speeds are alpha_s = max over the grid of
 * |lambda_s(u)| per field and direction, computed on the device, unless
 * alpha_host (HOST array of ndim*m values, [dir][field]) is given.
 * f: optional device array of caller-evaluated flux point values f(u_j), for
 * the 1D scalar case only; it then requires alpha_host (alpha = max|f'(u)|,
 * remark on flux splitting).  Moving side splits (WT_SIDES) are taken at the
 * context's time (wenotheta_set_sides).  Asynchronous. */
wt_status wenotheta_rhs(wt_ctx *ctx, const wt_grid *grid, const wt_params *prm,
                        const double *u, const double *f, const double *alpha_host,
                        double *L_out, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * right-hand side of wenotheta_rhs, same arguments and results (bit for bit),
 * without a context.  It calls no allocating routine: its scratch (the speed
 * slot, the error word and, for ndim > 1, the divergence accumulator of
 * m * ncell doubles) lives in a fixed device buffer of the library, 64 MiB per
 * GPU, held from the library's first use of that GPU until the process ends.
 *   - Runs on the current HIP device; stream must belong to it.  The first
 *     call on a device looks up the buffer's address there (no allocation,
 *     no stream work).
 *   - Size limit: for ndim > 1, m * ncell <= 8388096 (e.g. 2D Euler up to
 *     2097024 points, 1448^2); beyond it WT_ERR_SCRATCH is returned before
 *     any work is queued.  1D grids have no limit.
 *   - WT_SIDES grids are not supported (WT_ERR_UNSUPPORTED: there is no side
 *     table without a context); the default tile shapes are used.
 *   - status_dev: optional DEVICE int32 that receives, when the work has run,
 *     WT_OK or the error the device met (WT_ERR_NONPHYSICAL, WT_ERR_NONFINITE).
 *   - Every call on one GPU shares that GPU's buffer and leaves its contents
 *     there; each call clears what must start at zero.  Calls that overlap on
 *     one GPU (several streams, threads or processes' graphs at once) race and
 *     give undefined results: serialise them.
 * Asynchronous; argument errors are returned before any work is queued. */
wt_status wenotheta_rhs_noalloc(const wt_grid *grid, const wt_params *prm, const double *u,
                                const double *f, const double *alpha_host, double *L_out,
                                int32_t *status_dev, void *stream);

/* One 3-stage TVD Runge-Kutta step (Sec. 2.1) of u in place.  dt > 0 is used
 * as given; dt <= 0 selects the CFL step dt = cfl / sum_d(amax_d / dx_d),
 * amax_d the largest wave speed in direction d.  dt_used_dev: optional
 * DEVICE pointer receiving the step taken.  The step starts at the context's
 * time t and advances it to t + dt; its stages take moving side splits at
 * t, t + dt and t + dt/2.  Asynchronous. */
wt_status wenotheta_step(wt_ctx *ctx, const wt_grid *grid, const wt_params *prm,
                         double *u, double dt, double *dt_used_dev, void *stream);

/* Advance u in place from time t0 to t_end with CFL steps (Sec. 2.1 asks for
 * a proper CFL condition; the tests of Sec. 4.3 take CFL 0.5): each step takes
 * dt = cfl / sum_d(amax_d / dx_d) from the speeds of its initial state, the
 * last one clipped to end at t_end (a step that would leave less than 1e-6 of itself
 * to go is stretched to t_end), or until max_steps steps have been taken
 * (max_steps < 0: no limit).  Synchronises; *t_out and *steps_out (HOST,
 * optional) receive the time reached and the steps taken, which also becomes
 * the context's time.  Returns any error the device recorded. */
wt_status wenotheta_solve(wt_ctx *ctx, const wt_grid *grid, const wt_params *prm,
                          double *u, double t0, double t_end, int64_t max_steps,
                          double *t_out, int64_t *steps_out, void *stream);

/* Side table of the context for grids with bc[k] == WT_SIDES (sides[2k] the
 * lower and sides[2k + 1] the upper end of dimension k; entries of other
 * dimensions are not read), and the context's time t (HOST value, finite):
 * the time wenotheta_rhs takes moving splits at and wenotheta_step starts
 * from.  sides (HOST, 6 entries, copied) may be NULL to remove the table.
 * WT_ERR_ARG for an unknown kind, a NaN split0, a non-finite split_speed or a
 * non-finite entry of a given state (all 5, unused ones too); a given state that is not physical (rho <= 0 or
 * p <= 0) is reported by the device as WT_ERR_NONPHYSICAL when a ghost point
 * takes it.  Calls with WT_SIDES grids return WT_ERR_ARG while no table is
 * set.  Stream-ordered (the time is set on the stream). */
wt_status wenotheta_set_sides(wt_ctx *ctx, const wt_side *sides, double t, void *stream);

/* Batched solves: nprob independent 1D Euler problems (prm->system must be
 * WT_EULER, prm->gravity all 0, else WT_ERR_UNSUPPORTED) packed side by side
 * in one state, each advanced by nsteps CFL
 * steps of its own (dt_b = cfl / (amax_b / dx_b)), as one captured HIP graph:
 * by default one persistent kernel, or the flat form (one launch per stage
 * over all problems) where the batch tuner below chose it.
 *   u       DEVICE, FP64, [3][total] component-major: problem b occupies
 *           columns offset[b] .. offset[b] + n[b] - 1; advanced in place;
 *   n, offset, lo, hi, bc   HOST arrays of nprob entries: points (>= 6),
 *           first column, domain ends (dx_b = (hi - lo) / n) and boundary
 *           condition (any wt_bc) of each problem; the column ranges must be disjoint
 *           and inside [0, total);
 *   t_out      optional DEVICE array of nprob doubles: the time each problem
 *              reached;
 *   status_out optional DEVICE array of nprob int32: WT_OK, or
 *              WT_ERR_NONPHYSICAL / WT_ERR_NONFINITE for a problem whose
 *              state became non-physical (its columns of u are then
 *              unspecified; the other problems are unaffected).  Without
 *              status_out such an error is recorded in the context and
 *              returned by wenotheta_sync;
 *   steps_out  optional DEVICE array of nprob int64: the steps completed
 *              before a problem's state became non-physical (nsteps if it
 *              never did).
 * The WENO-theta step of each problem is the one wenotheta_step performs on
 * it alone (bit for bit in WT_FP64 and WT_FP64_FAST).  Asynchronous after the
 * problem tables are uploaded. */
wt_status wenotheta_solve_batched(wt_ctx *ctx, int64_t nprob, const int64_t *n,
                                  const int64_t *offset, const double *lo, const double *hi,
                                  const int32_t *bc, const wt_params *prm, double *u,
                                  int64_t total, int64_t nsteps, double *t_out,
                                  int32_t *status_out, int64_t *steps_out, void *stream);

/* Batched 2D solves: nprob independent 2D Euler problems of their own sizes
 * (dimension-by-dimension scheme of Sec. 4.3), packed side by side in one
 * state, each advanced by nsteps CFL steps of its own
 * (dt_b = cfl / (amax_x / dx_b + amax_y / dy_b)), as one captured HIP graph:
 * by default one persistent kernel in which one workgroup runs a whole
 * problem, or the flat form (one launch per pass over the tiles of all
 * problems) where the batch tuner below chose it.
 * prm->system must be WT_EULER and prm->gravity all 0 (else
 * WT_ERR_UNSUPPORTED).
 *   u       DEVICE, FP64, [4][total] component-major (rho, m_x, m_y, E):
 *           problem b occupies columns offset[b] .. offset[b] + nx[b] ny[b] - 1,
 *           its points x fastest (column offset[b] + y nx[b] + x); advanced in
 *           place;
 *   nx, ny, offset   HOST arrays of nprob entries: points per direction
 *           (>= 6 each, (nx + 1) ny and nx (ny + 1) at most 2^30) and first
 *           column; the column ranges must be disjoint and inside [0, total);
 *   lo, hi, bc       HOST arrays of 2 nprob entries, [problem][x, y]: domain
 *           ends (dx = (hi - lo) / n per direction) and boundary condition
 *           (any wt_bc) per direction;
 *   t_out, status_out, steps_out   as for wenotheta_solve_batched.
 * The step of each problem is the one wenotheta_step performs on it alone
 * (bit for bit in WT_FP64 and WT_FP64_FAST).  Asynchronous after the problem
 * tables are uploaded.  Calls on one context share the stage buffers of
 * wenotheta_solve_batched: the two must not overlap. */
wt_status wenotheta_solve_batched_2d(wt_ctx *ctx, int64_t nprob, const int64_t *nx,
                                     const int64_t *ny, const int64_t *offset, const double *lo,
                                     const double *hi, const int32_t *bc, const wt_params *prm,
                                     double *u, int64_t total, int64_t nsteps, double *t_out,
                                     int32_t *status_out, int64_t *steps_out, void *stream);

/* Tile variants of the batched kernels, chosen by timing (the batch form of
 * wenotheta_tune).  The variants compute the same operations, so results are
 * bit-identical whichever runs:
 *   1D batches: the persistent kernel with workgroups of 256 threads sweeping
 *               segments of 255 points (0, default) or of 128 threads and 127
 *               points (1), or the flat form (each stage one launch over the
 *               255-point segments of all problems) (2);
 *   2D batches: the persistent kernel with the x pass in tiles of 4 rows x 63
 *               points (0, default) or of 8 rows x 31 points (1), or the flat
 *               form (each pass one launch over the tiles of all problems, the
 *               problems' speeds, steps and errors in device arrays) with x tiles
 *               of 8 x 31 (2) or 4 x 63 (3) and the y pass in 8 columns x 31, or
 *               the flat form with packed chunks (4): each pass's interfaces of
 *               a problem listed line after line (rows; groups of 8 columns) and
 *               cut into chunks of 256 interfaces (x) or 32 interface rows of 8
 *               columns (y) overlapping by one, so that nearly every thread has
 *               an interface whatever the problem's size.
 * wenotheta_tune_batched / wenotheta_tune_batched_2d take the arguments of the
 * corresponding solve (u DEVICE, only read: each variant runs probe_steps >= 1
 * steps on a scratch copy, 3 rounds interleaved, the best launch kept), keep
 * the fastest variant in the context for batches with the same sizes, layout
 * and precision (the default stays unless another is more than 2% faster) and
 * write it to *variant_out (HOST, optional).  Synchronises the stream;
 * allocates and frees its scratch copy.
 * wenotheta_set_batched_tiles forces variant (1D: 0 to 2; 2D: 0 to 4) for every
 * later batch of ndim (1 or 2) dimensions on this context. */
wt_status wenotheta_tune_batched(wt_ctx *ctx, int64_t nprob, const int64_t *n,
                                 const int64_t *offset, const double *lo, const double *hi,
                                 const int32_t *bc, const wt_params *prm, const double *u,
                                 int64_t total, int64_t probe_steps, int32_t *variant_out,
                                 void *stream);
wt_status wenotheta_tune_batched_2d(wt_ctx *ctx, int64_t nprob, const int64_t *nx,
                                    const int64_t *ny, const int64_t *offset, const double *lo,
                                    const double *hi, const int32_t *bc, const wt_params *prm,
                                    const double *u, int64_t total, int64_t probe_steps,
                                    int32_t *variant_out, void *stream);
wt_status wenotheta_set_batched_tiles(wt_ctx *ctx, int32_t ndim, int32_t variant);

/* Tile shapes of the sweeps (dimension-by-dimension scheme of Sec. 4.3: one
 * 1D operator per direction), 256 interfaces per workgroup.  The y and z
 * sweeps of the 2D/3D Euler system run in one of four tile shapes, TX
 * consecutive x-columns by TN points along the sweep direction:
 *   0: 8 x 31 (default)   1: 16 x 15   2: 4 x 63   3: 32 x 7
 * and their x sweeps in one of two, rows by TN points along x:
 *   0: 1 x 255 (default)  1: 8 x 31 (for rows that 255-point segments would
 *                          leave a nearly empty last segment, e.g. 512 points)
 * or, for the 2D Euler system without WT_SIDES dimensions, x variant
 *   2: the fused stage kernel: both directions of a stage in one launch on
 *      tiles of 31 x 15 points with 3-point halos, so that the divergence of
 *      the x direction stays on chip (the y entry is then unused)
 * Every shape computes the same fluxes with the same operations: the results
 * are bit-identical whichever is used; only the speed differs.  The choice
 * is kept in the context per grid shape (system, ndim, n, precision; the 16
 * most recent shapes).
 *
 * wenotheta_tune times each shape on `u` (DEVICE, the state layout of
 * wenotheta_rhs; only read) with the sweep that writes the context's
 * workspace, keeps the fastest, and writes it to tile_out[0..ndim-1] (HOST,
 * optional; entry 0 is the x sweep's).  The context's time is left
 * as it was.  It synchronises `stream` (do not call it during graph capture)
 * and returns any device error.
 *
 * wenotheta_set_tiles sets the shapes for the grid instead: tile[0] in 0..1
 * (0..2 for the 2D Euler system without WT_SIDES dimensions) and tile[d] in
 * 0..3 for 0 < d < ndim (HOST); systems or dimensions without choices (scalar
 * laws, 1D) ignore the entries.  No device work. */
wt_status wenotheta_tune(wt_ctx *ctx, const wt_grid *grid, const wt_params *prm, const double *u,
                         int32_t *tile_out, void *stream);
wt_status wenotheta_set_tiles(wt_ctx *ctx, const wt_grid *grid, const wt_params *prm,
                              const int32_t *tile);

/* Wait for the work queued on `stream` and return (and clear) any error the
 * device recorded since the last synchronising call. */
wt_status wenotheta_sync(wt_ctx *ctx, void *stream);

/* Per-kernel timing.  enable != 0 starts recording a pair of HIP events on the
 * launch stream around every sweep kernel (and clears the totals); 0 stops.
 * Measurement support for callers that report kernel durations; it does not
 * change any result. */
wt_status wenotheta_profile(wt_ctx *ctx, int32_t enable);

/* Totals since wenotheta_profile(ctx, 1), folded in at each synchronising
 * call: ms[k] (HOST) the summed kernel milliseconds and count[k] (HOST) the
 * launches of kind k for k < min(nkinds, 7), nkinds >= 6.  Kind d (0..2) is the
 * sweep along direction d in a non-final role (writing or accumulating the
 * divergence); kind 3 + d is the sweep along d that finishes a stage or an RHS
 * evaluation; kind 6 is the fused 2D stage kernel.
 * Returns WT_ERR_ARG if more launches were queued between two synchronising
 * calls than could be recorded (4096). */
wt_status wenotheta_profile_read(wt_ctx *ctx, double *ms, int64_t *count, int32_t nkinds);

#ifdef __cplusplus
}
#endif
#endif /* WENOTHETA_H */
