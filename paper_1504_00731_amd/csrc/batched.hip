// Batched solves: many independent 1D or 2D Euler problems of uneven sizes
// advanced by one persistent kernel.
//
// Each workgroup takes a problem from a work queue (largest first), and runs
// all of that problem's RK3 steps itself: per stage it sweeps the problem in
// segments of 255 points (the same staged-tile / one-interface-per-thread /
// flux-difference structure as the grid sweeps), writing the next stage state;
// the problem's Lax-Friedrichs speeds and its CFL step are block reductions,
// so no grid-wide synchronisation is ever needed.  The stage buffers of a
// problem are touched by one workgroup only; a device-scope fence and a
// barrier separate a stage's writes from the next stage's reads.  The whole
// batch is one graph (queue reset + kernel), captured once per argument set
// and replayed.
//
// 2D problems take per stage an x pass over tiles of 4 rows x 63 points
// (divergence of the x fluxes into a packed workspace D) and a y pass over
// tiles of 8 columns x 31 points (L = -(D + y divergence), the stage update and
// the new speeds), with the grid sweeps' staging, interface routine and
// operation order; both tile shapes pack several rows or columns, so a short
// line does not leave most of the 256 threads idle.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <vector>

#include "wenotheta.h"
#include "wt_ctx.hpp"
#include "wt_device.hpp"
#include "wt_pack.hpp"

namespace wt {

struct BatchArgs {
    double *u;                 // packed states [3][total], advanced in place
    double *U1, *U2;           // packed stage buffers
    int64_t total;
    // flat form: segment table and the per-problem state
    const int32_t *ft_prob, *ft_local;
    int64_t nft;
    unsigned long long *f_spd;
    double *f_dt, *f_time;
    int32_t *f_err;
    int64_t *f_first;
    const int64_t *n, *off;    // points and first column of each problem
    const double *dx, *rdx;    // spacing and its rounded reciprocal
    const int32_t *bc;         // boundary condition of each problem
    const int32_t *order;      // problems, largest first
    int32_t *queue;            // next queue position
    double *t_out;             // time reached per problem (optional)
    int32_t *status_out;       // status per problem (optional)
    int64_t *steps_out;        // steps completed per problem (optional)
    DevState *st;
    int nprob;
    int64_t nsteps;
    double gamma, cfl;
    WenoConst W;
};

// Block-wide max of K per-thread values over NW waves; every thread gets the result.
template <int K, int NW>
__device__ __forceinline__ void block_max(double (&v)[K], double (*red)[NW])
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double w = wave_max_to_lane63(v[k]);
        if (lane == 63) red[k][wid] = w;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double m = red[k][0];
#pragma unroll
        for (int w = 1; w < NW; ++w) m = red[k][w] > m ? red[k][w] : m;
        v[k] = m;
    }
    __syncthreads();
}

// A value every lane of the wave holds alike, read once as a scalar (it then
// lives in scalar registers instead of one vector register pair per lane).
__device__ __forceinline__ double uniform(double x)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}


// The FP64 form is held to 3 waves per SIMD (at most 168 VGPRs): left to
// itself it takes 174, and it fits 164 without spilling.  The FP32 form
// reaches 3 waves by itself.
// Workgroups of TPB threads sweep a problem in segments of TPB - 1 points (the
// tile variants the batch tuner chooses between: 256 and 128 threads).  The FP64
// form recomputes the rows of L and columns of R per field and runs at 4 waves per
// SIMD (a small spill outside the interface loop; 2% faster than 3 waves); the FP32
// form keeps them and runs at 3 (at 4 it spilled inside the loop, 14% slower).
template <int PREC, int TPB>
__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(PREC == 0 ? 4 : 3)))
void batched_kernel(BatchArgs A)
{
    constexpr int M = 3, TN = TPB - 1, NC = TN + 6, NW = TPB / 64;
    constexpr bool FAST = PREC == 2;        // the fast FP64 cell and stage forms
    __shared__ double s_u[M][NC];
    __shared__ double s_f[M][NC];
    __shared__ double s_v[1][NC];
    __shared__ double s_sr[NC];
    __shared__ double s_H[NC];
    __shared__ double s_F[M][TPB];
    __shared__ double s_red[3][NW];
    __shared__ double s_al[3];
    __shared__ int s_job;
    __shared__ int s_bad;
    __shared__ unsigned long long s_first;

    const int t = threadIdx.x;
    const int64_t total = A.total;
    // The job loop's control flow is kept wave-uniform: the job index is read
    // once per wave as a scalar, so its exit and every loop bound below are
    // uniform branches, and a barrier closes each job after thread 0's tail, so
    // that tail and the next fetch (both on thread 0 alone) stay separate blocks.
    // Were they merged into one thread-0 path around the loop, the other lanes
    // of wave 0 would return to the fetch barrier without thread 0 and re-read
    // a stale job index for ever.
    for (;;) {
        if (t == 0) s_job = atomicAdd(A.queue, 1);
        __syncthreads();
        const int job = __builtin_amdgcn_readfirstlane(s_job);
        if (job >= A.nprob) break;              // every workgroup leaves once the queue is empty
        const int b = A.order[job];
        const int64_t n = A.n[b], off = A.off[b];
        const double dx = A.dx[b], rdx = A.rdx[b];
        const int bc = A.bc[b];
        const int64_t nseg = (n + TN - 1) / TN;
        int err = 0;

        // speeds of the initial state
        double spd[3] = {0.0, 0.0, 0.0};
        for (int64_t i = t; i < n; i += TPB) {
            double uc[3] = {A.u[off + i], A.u[total + off + i], A.u[2 * total + off + i]};
            double lam[3];
            err |= euler_speeds<1>(uc, A.gamma, lam);
#pragma unroll
            for (int k = 0; k < 3; ++k) spd[k] = lam[k] > spd[k] ? lam[k] : spd[k];
        }
        block_max<3, NW>(spd, s_red);
#pragma unroll
        for (int k = 0; k < 3; ++k) spd[k] = uniform(spd[k]);

        double time = 0.0;
        // first step at which this thread met a non-physical state (nsteps: none)
        int64_t first_bad = err ? 0 : A.nsteps;
        for (int64_t step = 0; step < A.nsteps; ++step) {
            // dt = cfl / (amax / dx), amax = max(|u| + c) = max(alpha_0, alpha_2)
            const double am = spd[2] > spd[0] ? spd[2] : spd[0];
            const double dt = uniform(div_rn(A.cfl, div_rn(am, dx)));
            for (int stage = 1; stage <= 3; ++stage) {
                const double *uin = stage == 1 ? A.u : (stage == 2 ? A.U1 : A.U2);
                double *out = stage == 1 ? A.U1 : (stage == 2 ? A.U2 : A.u);
                if (t < 3)
                    s_al[t] = split_speed([&spd](int k) { return spd[k]; }, t, bc == WT_REFLECTIVE);
                // the new state's speeds: per-wave maxima over the segments, in LDS
                if ((t & 63) < 3) s_red[t & 63][t >> 6] = 0.0;
                for (int64_t seg = 0; seg < nseg; ++seg) {
                    const int64_t g0 = seg * TN;
                    // stage the segment and its halos
                    for (int i = t; i < NC; i += TPB) {
                        const int64_t g = map_index(g0 - 3 + i, n, bc);
                        double uc[3];
#pragma unroll
                        for (int c = 0; c < 3; ++c) uc[c] = uin[c * total + off + g];
                        if (reflected(g0 - 3 + i, n, bc)) uc[1] = -uc[1];
                        double vel[1], p, H;
                        if (!euler_cell<1, FAST>(uc, A.gamma, vel, p, H)) {
                            const bool fin = __builtin_isfinite(uc[0]) && __builtin_isfinite(uc[1]) &&
                                             __builtin_isfinite(uc[2]);
                            err |= fin ? kErrNonphysical : kErrNonfinite;
                        }
#pragma unroll
                        for (int c = 0; c < 3; ++c) s_u[c][i] = uc[c];
                        if constexpr (fast_math<PREC>()) {
                            s_f[0][i] = p;      // the fast forms project the flux from p
                        } else {
                            double fn[3];
                            euler_normal_flux<1, 0>(uc, vel, p, fn);
#pragma unroll
                            for (int c = 0; c < 3; ++c) s_f[c][i] = fn[c];
                        }
                        s_v[0][i] = vel[0];
                        s_sr[i] = FAST ? sqrt_fast(uc[0]) : sqrt_rn(uc[0]);
                        s_H[i] = H;
                    }
                    __syncthreads();
                    if (g0 + t <= n) {
                        const LdsStencil<M, 1, NC, 1, fast_math<PREC>()> S{s_u, s_f, s_v, s_sr, s_H, t,
                                                                           &s_f[0][0]};
                        double F[3];
                        if (!euler_interface_flux<1, 0, PREC, PREC == 0>(S, LdsSpeeds{s_al}, A.gamma, A.W, F))
                            err |= kErrNonphysical;
#pragma unroll
                        for (int c = 0; c < 3; ++c) s_F[c][t] = F[c];
                    }
                    __syncthreads();
                    double lam[3] = {0.0, 0.0, 0.0};
                    if (t < TN && g0 + t < n) {
                        const int64_t idx = off + g0 + t;
                        double u0v[3];
                        stage_u0<3>(stage, A.u, total, idx, u0v);
                        double un[3];
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            const double L = -flux_quotient<FAST>(s_F[c][t + 1] - s_F[c][t], dx, rdx);
                            const int64_t o = c * total + idx;
                            un[c] = rk3_stage<FAST>(stage, uin[o], L, dt, u0v[c]);
                        }
#pragma unroll
                        for (int c = 0; c < 3; ++c) out[c * total + idx] = un[c];
                        err |= euler_speeds<1, FAST>(un, A.gamma, lam);
                    }
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        const double w = wave_max_to_lane63(lam[k]);
                        if ((t & 63) == 63) s_red[k][t >> 6] = w > s_red[k][t >> 6] ? w : s_red[k][t >> 6];
                    }
                    __syncthreads();                // the tile is reused by the next segment
                }
                // the next stage reads what this one wrote
                __threadfence();
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    double m = s_red[k][0];
#pragma unroll
                    for (int w = 1; w < NW; ++w) m = s_red[k][w] > m ? s_red[k][w] : m;
                    spd[k] = uniform(m);
                }
                __syncthreads();                    // s_red is cleared again by the next stage
            }
            if (err && first_bad == A.nsteps) first_bad = step;
            time = uniform(time + dt);
        }
        // per-problem outcome (a failed problem keeps being advanced; its columns are
        // then unspecified): OR of the error bits and the first failing step
        if (t == 0) {
            s_bad = 0;
            s_first = A.nsteps;
        }
        __syncthreads();
        if (err) atomicOr(&s_bad, err);
        if (first_bad < A.nsteps) atomicMin(&s_first, (unsigned long long)first_bad);
        __syncthreads();
        if (t == 0) {
            const int all_err = s_bad;
            if (A.t_out) A.t_out[b] = time;
            if (A.steps_out) A.steps_out[b] = (int64_t)s_first;
            if (A.status_out)
                A.status_out[b] = all_err & kErrNonfinite ? WT_ERR_NONFINITE
                                                          : (all_err ? WT_ERR_NONPHYSICAL : WT_OK);
            else if (all_err)
                atomicOr(&A.st->err, all_err);
        }
        // s_job, s_bad and s_first are rewritten by thread 0 only after this
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// 2D problems
// ---------------------------------------------------------------------------

// One 2D problem of a batch: nx x ny points (x fastest) from column off of the
// packed arrays, spacings with their rounded reciprocals, boundary conditions.
struct Prob2 {
    int64_t nx, ny, off;
    double dx, rdx, dy, rdy;
    int32_t bcx, bcy;
};

struct Batch2Args {
    double *u;                 // packed states [4][total], advanced in place
    double *U1, *U2, *D;       // packed stage buffers and the x divergence
    int64_t total;
    const Prob2 *prob;
    // flat form: per-pass tile tables (x pass in 8 x 31 and 4 x 63 tiles, y pass in
    // 8 x 31) and the per-problem state
    const int32_t *xt_prob[2], *xt_local[2], *yt_prob, *yt_local;
    int64_t ntx[2], nty;
    // packed tiles (variant 4): per pass (x, y) the problem, first interface and
    // interface count of each chunk
    const int32_t *pk_prob[2], *pk_q0[2], *pk_n[2];
    int64_t npk[2];
    unsigned long long *f_spd;
    double *f_dt, *f_time;
    int32_t *f_err;
    int64_t *f_first;
    const int32_t *order;      // problems, largest first
    int32_t *queue;            // next queue position
    double *t_out;             // time reached per problem (optional)
    int32_t *status_out;       // status per problem (optional)
    int64_t *steps_out;        // steps completed per problem (optional)
    DevState *st;
    int nprob;
    int64_t nsteps;
    double gamma, cfl;
    WenoConst W;
};

// Tile of a 2D problem: TX lines (rows for DIR 0, columns for DIR 1), each with
// TN owned points along DIR and 3-point halos mapped through the boundary; entry
// r * TX + l holds point g0 - 3 + r of line l0 + l (lines past the last repeat
// it; their interfaces are never taken).  Returns error bits.
template <int DIR, int TX, int TN, int NC, bool FAST, bool PRESS>
__device__ __forceinline__ int stage_tile2(const double *uin, int64_t total, const Prob2 &P,
                                           int64_t l0, int64_t g0, double gamma,
                                           double (*s_u)[NC], double (*s_f)[NC],
                                           double (*s_v)[NC], double *s_sr, double *s_H)
{
    constexpr int M = 4;
    const int64_t nd = DIR == 0 ? P.nx : P.ny, nl = DIR == 0 ? P.ny : P.nx;
    const int bc = DIR == 0 ? P.bcx : P.bcy;
    int err = 0;
    for (int i = threadIdx.x; i < (TN + 6) * TX; i += kThreads) {
        const int r = i / TX, cl = i % TX;
        const int64_t g = map_index(g0 - 3 + r, nd, bc);
        const int64_t l = l0 + cl < nl ? l0 + cl : nl - 1;
        const int64_t idx = P.off + (DIR == 0 ? l * P.nx + g : g * P.nx + l);
        double uc[M];
#pragma unroll
        for (int c = 0; c < M; ++c) uc[c] = uin[c * total + idx];
        if (reflected(g0 - 3 + r, nd, bc)) uc[1 + DIR] = -uc[1 + DIR];
        double vel[2], p, H;
        if (!euler_cell<2, FAST>(uc, gamma, vel, p, H)) {
            bool fin = true;
#pragma unroll
            for (int c = 0; c < M; ++c) fin = fin && __builtin_isfinite(uc[c]);
            err |= fin ? kErrNonphysical : kErrNonfinite;
        }
#pragma unroll
        for (int c = 0; c < M; ++c) s_u[c][i] = uc[c];
        if constexpr (PRESS) {
            s_f[0][i] = p;                  // the fast forms project the flux from p
        } else {
            double fn[M];
            euler_normal_flux<2, DIR>(uc, vel, p, fn);
#pragma unroll
            for (int c = 0; c < M; ++c) s_f[c][i] = fn[c];
        }
        s_v[0][i] = vel[0];
        s_v[1][i] = vel[1];
        s_sr[i] = FAST ? sqrt_fast(uc[0]) : sqrt_rn(uc[0]);
        s_H[i] = H;
    }
    return err;
}

// Interface fluxes of a staged tile, one interface per thread (between points
// g0 + it - 1 and g0 + it of line l0 + l, t = it * TX + l), into s_F.
// With ALIAS, s_F overlays s_f: the fluxes are stored after a barrier that
// closes every thread's stencil reads.
template <int DIR, int TX, int TN, int NC, int PREC, bool ALIAS = false>
__device__ __forceinline__ int tile_fluxes2(const Prob2 &P, int64_t l0, int64_t g0, const double *al,
                                            double gamma, const WenoConst &W,
                                            const double (*s_u)[NC], const double (*s_f)[NC],
                                            const double (*s_v)[NC], const double *s_sr,
                                            const double *s_H, double (*s_F)[kThreads])
{
    const int t = threadIdx.x, it = t / TX, cl = t % TX;
    const int64_t nd = DIR == 0 ? P.nx : P.ny, nl = DIR == 0 ? P.ny : P.nx;
    int err = 0;
    const bool valid = l0 + cl < nl && g0 + it <= nd;
    double F[4];
    if (valid) {
        const LdsStencil<4, 2, NC, TX, fast_math<PREC>()> S{s_u, s_f, s_v, s_sr, s_H, t, &s_f[0][0]};
        if (!euler_interface_flux<2, DIR, PREC, true>(S, LdsSpeeds{al}, gamma, W, F)) err = kErrNonphysical;
    }
    if constexpr (ALIAS) __syncthreads();
    if (valid) {
#pragma unroll
        for (int q = 0; q < 4; ++q) s_F[q][t] = F[q];
    }
    return err;
}

// Tile variants the batch tuner chooses between: the x pass in tiles of 4 rows x 63
// points (XV = 0) or 8 rows x 31 points (XV = 1); the y pass in 8 columns x 31.
// Rows of L and columns of R are recomputed per field (fewer registers live across
// the field loop: the FP64 form's spill falls from 84 to 28 bytes at 3 waves).
template <int PREC, int XV>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3)))
void batched2d_kernel(Batch2Args A)
{
    constexpr int M = 4, XTX = XV == 0 ? 4 : 8, XTN = XV == 0 ? 63 : 31, YTX = 8, YTN = 31;
    constexpr bool FAST = PREC == 2;        // the fast FP64 cell and stage forms
    constexpr int NC = (YTN + 6) * YTX > (XTN + 6) * XTX ? (YTN + 6) * YTX : (XTN + 6) * XTX;
    static_assert(XTX * (XTN + 1) == kThreads && YTX * (YTN + 1) == kThreads, "one interface per thread");
    __shared__ double s_u[M][NC];
    __shared__ double s_f[M][NC];
    __shared__ double s_v[2][NC];
    __shared__ double s_sr[NC];
    __shared__ double s_H[NC];
    __shared__ double s_F[M][kThreads];
    __shared__ double s_red[6][kThreads / 64];
    __shared__ double s_al[2][M];
    __shared__ int s_job;
    __shared__ int s_bad;
    __shared__ unsigned long long s_first;

    const int t = threadIdx.x;
    const int64_t total = A.total;
    // wave-uniform job loop, as in the 1D kernel
    for (;;) {
        if (t == 0) s_job = atomicAdd(A.queue, 1);
        __syncthreads();
        const int job = __builtin_amdgcn_readfirstlane(s_job);
        if (job >= A.nprob) break;
        const Prob2 P = A.prob[A.order[job]];
        const int b = A.order[job];
        const int64_t ncell = P.nx * P.ny;
        int err = 0;

        // speeds of the initial state: per direction |u_d - c|, |u_d|, |u_d + c|
        double spd[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int64_t i = t; i < ncell; i += kThreads) {
            double uc[M];
#pragma unroll
            for (int c = 0; c < M; ++c) uc[c] = A.u[c * total + P.off + i];
            double lam[6];
            err |= euler_speeds<2>(uc, A.gamma, lam);
#pragma unroll
            for (int k = 0; k < 6; ++k) spd[k] = lam[k] > spd[k] ? lam[k] : spd[k];
        }
        block_max<6, kThreads / 64>(spd, s_red);
#pragma unroll
        for (int k = 0; k < 6; ++k) spd[k] = uniform(spd[k]);

        const int64_t xlines = (P.ny + XTX - 1) / XTX, xseg = (P.nx + XTN - 1) / XTN;
        const int64_t ylines = (P.nx + YTX - 1) / YTX, yseg = (P.ny + YTN - 1) / YTN;
        double time = 0.0;
        int64_t first_bad = err ? 0 : A.nsteps;
        for (int64_t step = 0; step < A.nsteps; ++step) {
            // dt = cfl / (amax_x / dx + amax_y / dy), amax_d = max(alpha_{d,0}, alpha_{d,2})
            const double ax = spd[2] > spd[0] ? spd[2] : spd[0];
            const double ay = spd[5] > spd[3] ? spd[5] : spd[3];
            const double dt = uniform(div_rn(A.cfl, div_rn(ax, P.dx) + div_rn(ay, P.dy)));
            for (int stage = 1; stage <= 3; ++stage) {
                const double *uin = stage == 1 ? A.u : (stage == 2 ? A.U1 : A.U2);
                double *out = stage == 1 ? A.U1 : (stage == 2 ? A.U2 : A.u);
                // split speeds of each direction and field (the shear field takes |u_d|)
                if (t == 0) {
#pragma unroll
                    for (int d = 0; d < 2; ++d) {
                        const bool walls = (d == 0 ? P.bcx : P.bcy) == WT_REFLECTIVE;
#pragma unroll
                        for (int f = 0; f < M; ++f)
                            s_al[d][f] = split_speed([&spd, d](int k) { return spd[3 * d + (k < 3 ? k : 1)]; },
                                                     f, walls);
                    }
                }
                if ((t & 63) < 6) s_red[t & 63][t >> 6] = 0.0;

                // x pass: D = x divergence
                for (int64_t tile = 0; tile < xlines * xseg; ++tile) {
                    const int64_t l0 = (tile / xseg) * XTX, g0 = (tile % xseg) * XTN;
                    err |= stage_tile2<0, XTX, XTN, NC, FAST, fast_math<PREC>()>(uin, total, P, l0, g0, A.gamma, s_u, s_f, s_v, s_sr, s_H);
                    __syncthreads();
                    err |= tile_fluxes2<0, XTX, XTN, NC, PREC>(P, l0, g0, s_al[0], A.gamma, A.W, s_u, s_f,
                                                                s_v, s_sr, s_H, s_F);
                    __syncthreads();
                    if (t < XTN * XTX) {
                        const int it = t / XTX, cl = t % XTX;
                        const int64_t g = g0 + it, l = l0 + cl;
                        if (l < P.ny && g < P.nx) {
                            const int64_t idx = P.off + l * P.nx + g;
#pragma unroll
                            for (int c = 0; c < M; ++c)
                                A.D[c * total + idx] = flux_quotient<FAST>(s_F[c][t + XTX] - s_F[c][t], P.dx, P.rdx);
                        }
                    }
                    __syncthreads();                // the tile is reused by the next one
                }
                // the y pass reads what the x pass wrote
                __threadfence();
                __syncthreads();

                // y pass: L = -(D + y divergence), the stage, the new speeds
                for (int64_t tile = 0; tile < ylines * yseg; ++tile) {
                    const int64_t l0 = (tile / yseg) * YTX, g0 = (tile % yseg) * YTN;
                    err |= stage_tile2<1, YTX, YTN, NC, FAST, fast_math<PREC>()>(uin, total, P, l0, g0, A.gamma, s_u, s_f, s_v, s_sr, s_H);
                    __syncthreads();
                    err |= tile_fluxes2<1, YTX, YTN, NC, PREC>(P, l0, g0, s_al[1], A.gamma, A.W, s_u, s_f,
                                                                s_v, s_sr, s_H, s_F);
                    __syncthreads();
                    double lam[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                    if (t < YTN * YTX) {
                        const int it = t / YTX, cl = t % YTX;
                        const int64_t g = g0 + it, l = l0 + cl;
                        if (l < P.nx && g < P.ny) {
                            const int64_t idx = P.off + g * P.nx + l;
                            double u0v[M];
                            stage_u0<M>(stage, A.u, total, idx, u0v);
                            double un[M];
#pragma unroll
                            for (int c = 0; c < M; ++c) {
                                const int64_t o = c * total + idx;
                                const double Dd = flux_quotient<FAST>(s_F[c][t + YTX] - s_F[c][t], P.dy, P.rdy);
                                const double L = -(A.D[o] + Dd);
                                un[c] = rk3_stage<FAST>(stage, uin[o], L, dt, u0v[c]);
                            }
#pragma unroll
                            for (int c = 0; c < M; ++c) out[c * total + idx] = un[c];
                            err |= euler_speeds<2, FAST>(un, A.gamma, lam);
                        }
                    }
#pragma unroll
                    for (int k = 0; k < 6; ++k) {
                        const double w = wave_max_to_lane63(lam[k]);
                        if ((t & 63) == 63) s_red[k][t >> 6] = w > s_red[k][t >> 6] ? w : s_red[k][t >> 6];
                    }
                    __syncthreads();                // the tile is reused by the next one
                }
                // the next stage reads what this one wrote
                __threadfence();
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    double m = s_red[k][0];
#pragma unroll
                    for (int w = 1; w < kThreads / 64; ++w) m = s_red[k][w] > m ? s_red[k][w] : m;
                    spd[k] = uniform(m);
                }
                __syncthreads();                    // s_red and s_al are rewritten by the next stage
            }
            if (err && first_bad == A.nsteps) first_bad = step;
            time = uniform(time + dt);
        }
        if (t == 0) {
            s_bad = 0;
            s_first = A.nsteps;
        }
        __syncthreads();
        if (err) atomicOr(&s_bad, err);
        if (first_bad < A.nsteps) atomicMin(&s_first, (unsigned long long)first_bad);
        __syncthreads();
        if (t == 0) {
            const int all_err = s_bad;
            if (A.t_out) A.t_out[b] = time;
            if (A.steps_out) A.steps_out[b] = (int64_t)s_first;
            if (A.status_out)
                A.status_out[b] = all_err & kErrNonfinite ? WT_ERR_NONFINITE
                                                          : (all_err ? WT_ERR_NONPHYSICAL : WT_OK);
            else if (all_err)
                atomicOr(&A.st->err, all_err);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// 2D problems, flat form: every pass is one launch over the tiles of all
// problems (tile -> problem from a table), with the problems' Lax-Friedrichs
// speeds, time steps and error flags in per-problem device arrays; one step is
// a time-step kernel and an x and a y pass per stage.  The grid sweeps'
// occupancy instead of one workgroup per problem; the same tile routines and
// operation order, so each problem still equals its solve alone.
// ---------------------------------------------------------------------------

constexpr int kFlatSpeeds = 8;            // speeds per problem and slot (6 used)

struct Flat2Args {
    const double *uin, *u0;    // stage input, state at the start of the step
    double *out;               // stage output
    double *D;                 // x divergence
    int64_t total;
    const Prob2 *prob;
    const int32_t *tile_prob;  // problem of each tile (tiles listed problem by problem)
    const int32_t *tile_local; // index of the tile within its problem (packed: first interface)
    const int32_t *tile_count; // packed tiles: interfaces of the chunk
    int64_t ntiles, tiles_per_xcd;
    unsigned long long *spd;   // [3][nprob][kFlatSpeeds] speed slots (bits of doubles >= 0)
    double *dt;                // [nprob] time step of the current step
    double *time;              // [nprob] time reached
    int32_t *err;              // [nprob] error bits
    int64_t *first;            // [nprob] first step with an error (nsteps: none)
    int nprob;
    int rd, wr, zero;          // slots this stage reads, writes and clears
    int stage;                 // 1..3
    int64_t step, nsteps;
    double gamma, cfl;
    WenoConst W;
    double *t_out;
    int32_t *status_out;
    int64_t *steps_out;
    DevState *st;
};

__device__ __forceinline__ unsigned long long *flat_slot(const Flat2Args &A, int slot, int b)
{
    return A.spd + ((int64_t)slot * A.nprob + b) * kFlatSpeeds;
}

// Initial speeds of each problem (one workgroup per problem) into slot 0; slots
// 1 and 2 cleared; time, error flags and first failing step initialised.
__global__ __launch_bounds__(kThreads) void flat2_init_kernel(Flat2Args A)
{
    __shared__ double red[6][kThreads / 64];
    const int b = blockIdx.x;
    const Prob2 P = A.prob[b];
    const int64_t ncell = P.nx * P.ny;
    double spd[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int err = 0;
    for (int64_t i = threadIdx.x; i < ncell; i += kThreads) {
        double uc[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) uc[c] = A.uin[c * A.total + P.off + i];
        double lam[6];
        err |= euler_speeds<2>(uc, A.gamma, lam);
#pragma unroll
        for (int k = 0; k < 6; ++k) spd[k] = lam[k] > spd[k] ? lam[k] : spd[k];
    }
    block_max<6, kThreads / 64>(spd, red);
    __shared__ int s_err;
    if (threadIdx.x == 0) s_err = 0;
    __syncthreads();
    if (err) atomicOr(&s_err, err);
    __syncthreads();
    if (threadIdx.x < kFlatSpeeds) {
        const int k = threadIdx.x;
        flat_slot(A, 0, b)[k] = k < 6 ? double_to_bits(spd[k]) : 0ull;
        flat_slot(A, 1, b)[k] = 0ull;
        flat_slot(A, 2, b)[k] = 0ull;
    }
    if (threadIdx.x == 0) {
        A.time[b] = 0.0;
        A.err[b] = s_err;
        A.first[b] = s_err ? 0 : A.nsteps;
    }
}

// Start of step A.step: the first failing step of the step before, this
// step's dt (from the speeds of the step's initial state, slot 0) and the time
// after it, in the order of the persistent kernel.
__global__ void flat2_dt_kernel(Flat2Args A)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= A.nprob) return;
    if (A.step > 0 && A.err[b] && A.first[b] == A.nsteps) A.first[b] = A.step - 1;
    const Prob2 P = A.prob[b];
    const unsigned long long *sl = flat_slot(A, 0, b);
    const double l0 = bits_to_double(sl[0]), l2 = bits_to_double(sl[2]);
    const double l3 = bits_to_double(sl[3]), l5 = bits_to_double(sl[5]);
    const double ax = l2 > l0 ? l2 : l0;
    const double ay = l5 > l3 ? l5 : l3;
    const double dt = div_rn(A.cfl, div_rn(ax, P.dx) + div_rn(ay, P.dy));
    A.dt[b] = dt;
    A.time[b] = A.time[b] + dt;
}

// After the last step: outputs, like the persistent kernel's per-problem tail.
__global__ void flat2_finish_kernel(Flat2Args A)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= A.nprob) return;
    const int e = A.err[b];
    int64_t first = A.first[b];
    if (A.nsteps > 0 && e && first == A.nsteps) first = A.nsteps - 1;
    if (A.t_out) A.t_out[b] = A.time[b];
    if (A.steps_out) A.steps_out[b] = first;
    if (A.status_out)
        A.status_out[b] = e & kErrNonfinite ? WT_ERR_NONFINITE : (e ? WT_ERR_NONPHYSICAL : WT_OK);
    else if (e)
        atomicOr(&A.st->err, e);
}

// One pass (DIR 0: x, writing D; DIR 1: y, finishing the stage) over the tiles of
// all problems, tile shape TX x TN along DIR.
template <int DIR, int TX, int TN, int PREC>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(PREC == 0 ? 4 : 5)))
void flat2_pass_kernel(Flat2Args A)
{
    constexpr int M = 4, NC = (TN + 6) * TX;
    constexpr bool FAST = PREC == 2;        // the fast FP64 cell and stage forms
    static_assert(TX * (TN + 1) == kThreads && NC >= kThreads, "one interface per thread");
    __shared__ double s_u[M][NC];
    __shared__ double s_f[M][NC];
    __shared__ double s_v[2][NC];
    __shared__ double s_sr[NC];
    __shared__ double s_H[NC];
    // FP32: the interface fluxes take the rows of the staged normal fluxes (read by
    // no one once every interface is done), for a fifth workgroup per CU
    constexpr bool ALIAS_F = PREC != 0;
    __shared__ double s_Fown[ALIAS_F ? 1 : M][ALIAS_F ? 1 : kThreads];
    double (*s_F)[kThreads];
    if constexpr (ALIAS_F) s_F = reinterpret_cast<double (*)[kThreads]>(&s_f[0][0]);
    else s_F = reinterpret_cast<double (*)[kThreads]>(&s_Fown[0][0]);
    __shared__ double s_al[M];

    // block -> tile: each XCD takes a contiguous range of the table, so the tiles
    // of a problem (which share halo lines) meet in one L2
    int64_t tile = blockIdx.x;
    tile = (tile % kXcds) * A.tiles_per_xcd + tile / kXcds;
    if (tile >= A.ntiles) return;
    const int b = A.tile_prob[tile];
    const int local = A.tile_local[tile];
    const Prob2 P = A.prob[b];
    const int t = threadIdx.x;
    const int64_t nd = DIR == 0 ? P.nx : P.ny;
    const int64_t nseg = (nd + TN - 1) / TN;
    const int64_t l0 = (local / nseg) * TX, g0 = (local % nseg) * TN;

    // split speeds of this direction (the shear field takes |u_d|), paired at walls
    if (t == 0) {
        const unsigned long long *sl = flat_slot(A, A.rd, b);
        const bool walls = (DIR == 0 ? P.bcx : P.bcy) == WT_REFLECTIVE;
#pragma unroll
        for (int f = 0; f < M; ++f)
            s_al[f] = split_speed([sl](int k) { return bits_to_double(sl[3 * DIR + (k < 3 ? k : 1)]); },
                                  f, walls);
    }
    __builtin_amdgcn_s_setprio(2);      // staging at a raised issue priority (as the grid sweeps)
    int err = stage_tile2<DIR, TX, TN, NC, FAST, fast_math<PREC>()>(A.uin, A.total, P, l0, g0, A.gamma, s_u, s_f, s_v, s_sr, s_H);
    __builtin_amdgcn_s_setprio(0);
    __syncthreads();
    err |= tile_fluxes2<DIR, TX, TN, NC, PREC, ALIAS_F>(P, l0, g0, s_al, A.gamma, A.W, s_u, s_f, s_v, s_sr,
                                                         s_H, s_F);
    __syncthreads();
    const int it = t / TX, cl = t % TX;
    const int64_t g = g0 + it, l = l0 + cl;
    if constexpr (DIR == 0) {
        if (t < TN * TX && l < P.ny && g < P.nx) {
            const int64_t idx = P.off + l * P.nx + g;
#pragma unroll
            for (int c = 0; c < M; ++c)
                A.D[c * A.total + idx] = flux_quotient<FAST>(s_F[c][t + TX] - s_F[c][t], P.dx, P.rdx);
        }
        if (err) atomicOr(&A.err[b], err);
    } else {
        double lam[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (t < TN * TX && l < P.nx && g < P.ny) {
            const int64_t idx = P.off + g * P.nx + l;
            const double dt = A.dt[b];
            double u0v[M];
            stage_u0<M>(A.stage, A.u0, A.total, idx, u0v);
            double un[M];
#pragma unroll
            for (int c = 0; c < M; ++c) {
                const int64_t o = c * A.total + idx;
                const double Dd = flux_quotient<FAST>(s_F[c][t + TX] - s_F[c][t], P.dy, P.rdy);
                const double L = -(A.D[o] + Dd);
                un[c] = rk3_stage<FAST>(A.stage, A.uin[o], L, dt, u0v[c]);
            }
#pragma unroll
            for (int c = 0; c < M; ++c) A.out[c * A.total + idx] = un[c];
            err |= euler_speeds<2, FAST>(un, A.gamma, lam);
        }
        if (err) atomicOr(&A.err[b], err);
        // the new state's speeds: block maxima, one slot update per value
        int src[6], idx6[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            src[k] = k;
            idx6[k] = k;
        }
        // through the staged rows, free once every cell is updated (no lane moves)
        constexpr int KA = (M * NC) / kThreads < 6 ? (M * NC) / kThreads : 6;
        static_assert((6 - KA) * kThreads + 6 * 16 <= M * NC, "speed rows fit the staged rows");
        block_slot_max_lds<6, 6, kThreads, KA>(lam, flat_slot(A, A.wr, b), src, idx6, &s_u[0][0],
                                               &s_f[0][0]);
        if (local == 0 && t < kFlatSpeeds)
            __hip_atomic_store(&flat_slot(A, A.zero, b)[t], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Packed tiles of the flat 2D form (variant 4, wt_pack.hpp): a tile is a chunk of a
// problem's pass interfaces listed line after line, a line being a group of 8 rows (x
// pass) or 8 columns (y pass): 8 lanes by 32 interface rows, so that nearly every
// thread has an interface whatever the problem's size; the stretch of each line the
// chunk touches is staged with its halos.  A wave covers 8 interfaces along the pass
// in 8 lines, as the fixed 8 x 31 tiles do: near a jump across the lines only a few
// waves mix restricted and unrestricted stencils (a wave along one line of 64
// interfaces nearly always would, and pays for both).  The interface and cell
// routines are those of the other tiles, so results are bit-identical to them.
static_assert(kPackQt * kPackLanes == kThreads, "one interface per thread");

template <int DIR, int PREC>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(PREC == 0 ? 4 : 5)))
void flat2_packed_kernel(Flat2Args A)
{
    constexpr int M = 4, TX = kPackLanes;
    constexpr int NR = kPackRows, NC = NR * TX;
    constexpr bool FAST = PREC == 2;
    static_assert(NC >= kThreads, "the interface fluxes may overlay the staged normal fluxes");
    __shared__ double s_u[M][NC];
    __shared__ double s_f[M][NC];
    __shared__ double s_v[2][NC];
    __shared__ double s_sr[NC];
    __shared__ double s_H[NC];
    constexpr bool ALIAS_F = PREC != 0;
    __shared__ double s_Fown[ALIAS_F ? 1 : M][ALIAS_F ? 1 : kThreads];
    double (*s_F)[kThreads];
    if constexpr (ALIAS_F) s_F = reinterpret_cast<double (*)[kThreads]>(&s_f[0][0]);
    else s_F = reinterpret_cast<double (*)[kThreads]>(&s_Fown[0][0]);
    __shared__ double s_al[M];

    int64_t tile = blockIdx.x;
    tile = (tile % kXcds) * A.tiles_per_xcd + tile / kXcds;
    if (tile >= A.ntiles) return;
    const int b = A.tile_prob[tile];
    const int q0 = A.tile_local[tile], nq = A.tile_count[tile];
    const Prob2 P = A.prob[b];
    const int t = threadIdx.x;
    const int nd = (int)(DIR == 0 ? P.nx : P.ny);     // points along the pass
    const int64_t nlanes = DIR == 0 ? P.ny : P.nx;     // rows (x) or columns (y)
    const int W = nd + 1;                              // interfaces per line
    const int bc = DIR == 0 ? P.bcx : P.bcy;
    const int nrows = pack_rows(q0, nq, W);

    if (t == 0) {
        const unsigned long long *sl = flat_slot(A, A.rd, b);
        const bool walls = bc == WT_REFLECTIVE;
#pragma unroll
        for (int f = 0; f < M; ++f)
            s_al[f] = split_speed([sl](int k) { return bits_to_double(sl[3 * DIR + (k < 3 ? k : 1)]); },
                                  f, walls);
    }
    int err = 0;
    if (nrows > NR) {             // the host's chunk tables never ask for this
        if (t == 0) atomicOr(&A.err[b], kErrNonfinite);
        return;
    }
    // stage the lines' stretches: entry row * TX + lane
    __builtin_amdgcn_s_setprio(2);      // staging at a raised issue priority (as the grid sweeps)
    auto load_entry = [&](int e, double (&uc)[M]) {
        const int row = e / TX, lane = e % TX;
        int line, g;
        pack_point(q0, row, W, &line, &g);
        const int64_t gm = map_index(g, nd, bc);
        int64_t l = (int64_t)line * TX + lane;
        if (l >= nlanes) l = nlanes - 1;               // lanes past the last row/column repeat it
        const int64_t idx = P.off + (DIR == 0 ? l * P.nx + gm : gm * P.nx + l);
#pragma unroll
        for (int c = 0; c < M; ++c) uc[c] = A.uin[c * A.total + idx];
        if (reflected(g, nd, bc)) uc[1 + DIR] = -uc[1 + DIR];
    };
    auto convert_entry = [&](int e, const double (&uc)[M]) {
        double vel[2], p, H;
        if (!euler_cell<2, FAST>(uc, A.gamma, vel, p, H)) {
            bool fin = true;
#pragma unroll
            for (int c = 0; c < M; ++c) fin = fin && __builtin_isfinite(uc[c]);
            err |= fin ? kErrNonphysical : kErrNonfinite;
        }
#pragma unroll
        for (int c = 0; c < M; ++c) s_u[c][e] = uc[c];
        if constexpr (fast_math<PREC>()) {
            s_f[0][e] = p;                      // the fast forms project the flux from p
        } else {
            double fn[M];
            euler_normal_flux<2, DIR>(uc, vel, p, fn);
#pragma unroll
            for (int c = 0; c < M; ++c) s_f[c][e] = fn[c];
        }
        s_v[0][e] = vel[0];
        s_v[1][e] = vel[1];
        s_sr[e] = FAST ? sqrt_fast(uc[0]) : sqrt_rn(uc[0]);
        s_H[e] = H;
    };
    if constexpr (DIR == 0) {
        // the x pass loads both entries a thread stages before converting either (one
        // HBM latency before the barrier instead of two); the y pass, whose registers
        // are tighter, keeps the loop
        constexpr int NIT = (NC + kThreads - 1) / kThreads;
        double ucs[NIT][M];
#pragma unroll
        for (int it = 0; it < NIT; ++it)
            if (t + it * kThreads < nrows * TX) load_entry(t + it * kThreads, ucs[it]);
#pragma unroll
        for (int it = 0; it < NIT; ++it)
            if (t + it * kThreads < nrows * TX) convert_entry(t + it * kThreads, ucs[it]);
    } else {
        for (int e = t; e < nrows * TX; e += kThreads) {
            double uc[M];
            load_entry(e, uc);
            convert_entry(e, uc);
        }
    }
    __builtin_amdgcn_s_setprio(0);
    __syncthreads();
    // one interface per thread: interface row ir of the chunk, lane
    const int ir = t / TX, lane = t % TX;
    const int q = q0 + ir;
    const int line = q / W, i = q - line * W;
    const bool lane_ok = (int64_t)line * TX + lane < nlanes;
    double F[M];
    const bool valid = ir < nq && lane_ok;
    if (valid) {
        const LdsStencil<M, 2, NC, TX, fast_math<PREC>()> S{s_u, s_f, s_v, s_sr, s_H,
                                                            pack_base(q0, q, W) * TX + lane, &s_f[0][0]};
        if (!euler_interface_flux<2, DIR, PREC, true>(S, LdsSpeeds{s_al}, A.gamma, A.W, F))
            err |= kErrNonphysical;
    }
    if constexpr (ALIAS_F) __syncthreads();
    if (valid) {
#pragma unroll
        for (int c = 0; c < M; ++c) s_F[c][t] = F[c];
    }
    __syncthreads();
    // cells whose left interface is this thread's (not a line's last interface)
    const bool cell = ir < nq - 1 && i < nd && lane_ok;
    if constexpr (DIR == 0) {
        if (cell) {
            const int64_t idx = P.off + ((int64_t)line * TX + lane) * P.nx + i;
#pragma unroll
            for (int c = 0; c < M; ++c)
                A.D[c * A.total + idx] = flux_quotient<FAST>(s_F[c][t + TX] - s_F[c][t], P.dx, P.rdx);
        }
        if (err) atomicOr(&A.err[b], err);
    } else {
        double lam[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (cell) {
            const int64_t idx = P.off + (int64_t)i * P.nx + (int64_t)line * TX + lane;
            const double dt = A.dt[b];
            double u0v[M];
            stage_u0<M>(A.stage, A.u0, A.total, idx, u0v);
            double un[M];
#pragma unroll
            for (int c = 0; c < M; ++c) {
                const int64_t o = c * A.total + idx;
                const double Dd = flux_quotient<FAST>(s_F[c][t + TX] - s_F[c][t], P.dy, P.rdy);
                const double L = -(A.D[o] + Dd);
                un[c] = rk3_stage<FAST>(A.stage, A.uin[o], L, dt, u0v[c]);
            }
#pragma unroll
            for (int c = 0; c < M; ++c) A.out[c * A.total + idx] = un[c];
            err |= euler_speeds<2, FAST>(un, A.gamma, lam);
        }
        if (err) atomicOr(&A.err[b], err);
        int src[6], idx6[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            src[k] = k;
            idx6[k] = k;
        }
        // through the staged rows, free once every cell is updated (no lane moves)
        constexpr int KA = (M * NC) / kThreads < 6 ? (M * NC) / kThreads : 6;
        static_assert((6 - KA) * kThreads + 6 * 16 <= M * NC, "speed rows fit the staged rows");
        block_slot_max_lds<6, 6, kThreads, KA>(lam, flat_slot(A, A.wr, b), src, idx6, &s_u[0][0],
                                               &s_f[0][0]);
        if (q0 == 0 && t < kFlatSpeeds)
            __hip_atomic_store(&flat_slot(A, A.zero, b)[t], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ---------------------------------------------------------------------------
// 1D problems, flat form: the same organisation as the 2D flat form, one pass
// per stage over the 255-point segments of all problems.
// ---------------------------------------------------------------------------

constexpr int kFlat1Speeds = 4;           // speeds per problem and slot (3 used)

struct Flat1Args {
    const double *uin, *u0;    // stage input, state at the start of the step
    double *out;               // stage output
    int64_t total;
    const int64_t *n, *off;    // problem tables
    const double *dx, *rdx;
    const int32_t *bc;
    const int32_t *tile_prob, *tile_local;
    int64_t ntiles, tiles_per_xcd;
    unsigned long long *spd;   // [3][nprob][kFlat1Speeds]
    double *dt, *time;
    int32_t *err;
    int64_t *first;
    int nprob;
    int rd, wr, zero, stage;
    int64_t step, nsteps;
    double gamma, cfl;
    WenoConst W;
    double *t_out;
    int32_t *status_out;
    int64_t *steps_out;
    DevState *st;
};

__device__ __forceinline__ unsigned long long *flat1_slot(const Flat1Args &A, int slot, int b)
{
    return A.spd + ((int64_t)slot * A.nprob + b) * kFlat1Speeds;
}

__global__ __launch_bounds__(kThreads) void flat1_init_kernel(Flat1Args A)
{
    __shared__ double red[3][kThreads / 64];
    __shared__ int s_err;
    const int b = blockIdx.x;
    const int64_t n = A.n[b], off = A.off[b];
    double spd[3] = {0.0, 0.0, 0.0};
    int err = 0;
    for (int64_t i = threadIdx.x; i < n; i += kThreads) {
        double uc[3] = {A.uin[off + i], A.uin[A.total + off + i], A.uin[2 * A.total + off + i]};
        double lam[3];
        err |= euler_speeds<1>(uc, A.gamma, lam);
#pragma unroll
        for (int k = 0; k < 3; ++k) spd[k] = lam[k] > spd[k] ? lam[k] : spd[k];
    }
    block_max<3, kThreads / 64>(spd, red);
    if (threadIdx.x == 0) s_err = 0;
    __syncthreads();
    if (err) atomicOr(&s_err, err);
    __syncthreads();
    if (threadIdx.x < kFlat1Speeds) {
        const int k = threadIdx.x;
        flat1_slot(A, 0, b)[k] = k < 3 ? double_to_bits(spd[k]) : 0ull;
        flat1_slot(A, 1, b)[k] = 0ull;
        flat1_slot(A, 2, b)[k] = 0ull;
    }
    if (threadIdx.x == 0) {
        A.time[b] = 0.0;
        A.err[b] = s_err;
        A.first[b] = s_err ? 0 : A.nsteps;
    }
}

__global__ void flat1_dt_kernel(Flat1Args A)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= A.nprob) return;
    if (A.step > 0 && A.err[b] && A.first[b] == A.nsteps) A.first[b] = A.step - 1;
    const unsigned long long *sl = flat1_slot(A, 0, b);
    const double l0 = bits_to_double(sl[0]), l2 = bits_to_double(sl[2]);
    const double am = l2 > l0 ? l2 : l0;
    const double dt = div_rn(A.cfl, div_rn(am, A.dx[b]));
    A.dt[b] = dt;
    A.time[b] = A.time[b] + dt;
}

__global__ void flat1_finish_kernel(Flat1Args A)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= A.nprob) return;
    const int e = A.err[b];
    int64_t first = A.first[b];
    if (A.nsteps > 0 && e && first == A.nsteps) first = A.nsteps - 1;
    if (A.t_out) A.t_out[b] = A.time[b];
    if (A.steps_out) A.steps_out[b] = first;
    if (A.status_out)
        A.status_out[b] = e & kErrNonfinite ? WT_ERR_NONFINITE : (e ? WT_ERR_NONPHYSICAL : WT_OK);
    else if (e)
        atomicOr(&A.st->err, e);
}

// One stage over the 255-point segments of all problems.
template <int PREC>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4)))
void flat1_pass_kernel(Flat1Args A)
{
    constexpr int M = 3, TN = kThreads - 1, NC = TN + 6;
    constexpr bool FAST = PREC == 2;        // the fast FP64 cell and stage forms
    __shared__ double s_u[M][NC];
    __shared__ double s_f[M][NC];
    __shared__ double s_v[1][NC];
    __shared__ double s_sr[NC];
    __shared__ double s_H[NC];
    __shared__ double s_F[M][kThreads];
    __shared__ double s_al[M];

    int64_t tile = blockIdx.x;
    tile = (tile % kXcds) * A.tiles_per_xcd + tile / kXcds;
    if (tile >= A.ntiles) return;
    const int b = A.tile_prob[tile];
    const int64_t g0 = (int64_t)A.tile_local[tile] * TN;
    const int64_t n = A.n[b], off = A.off[b];
    const int bc = A.bc[b];
    const int t = threadIdx.x;
    if (t == 0) {
        const unsigned long long *sl = flat1_slot(A, A.rd, b);
#pragma unroll
        for (int f = 0; f < M; ++f)
            s_al[f] = split_speed([sl](int k) { return bits_to_double(sl[k]); }, f, bc == WT_REFLECTIVE);
    }
    int err = 0;
    __builtin_amdgcn_s_setprio(2);      // staging at a raised issue priority (as the grid sweeps)
    // both points a thread stages (NC > kThreads) loaded before either is converted, so
    // the block's barrier waits for one HBM latency, not two
    constexpr int NIT = (NC + kThreads - 1) / kThreads;
    double ucs[NIT][3];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int i = t + it * kThreads;
        if (i < NC) {
            const int64_t g = map_index(g0 - 3 + i, n, bc);
#pragma unroll
            for (int c = 0; c < 3; ++c) ucs[it][c] = A.uin[c * A.total + off + g];
            if (reflected(g0 - 3 + i, n, bc)) ucs[it][1] = -ucs[it][1];
        }
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int i = t + it * kThreads;
        if (i >= NC) continue;
        const double *uc = ucs[it];
        double vel[1], p, H;
        if (!euler_cell<1, FAST>(uc, A.gamma, vel, p, H)) {
            const bool fin = __builtin_isfinite(uc[0]) && __builtin_isfinite(uc[1]) && __builtin_isfinite(uc[2]);
            err |= fin ? kErrNonphysical : kErrNonfinite;
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) s_u[c][i] = uc[c];
        if constexpr (fast_math<PREC>()) {
            s_f[0][i] = p;                      // the fast forms project the flux from p
        } else {
            double fn[3];
            euler_normal_flux<1, 0>(uc, vel, p, fn);
#pragma unroll
            for (int c = 0; c < 3; ++c) s_f[c][i] = fn[c];
        }
        s_v[0][i] = vel[0];
        s_sr[i] = FAST ? sqrt_fast(uc[0]) : sqrt_rn(uc[0]);
        s_H[i] = H;
    }
    __builtin_amdgcn_s_setprio(0);
    __syncthreads();
    if (g0 + t <= n) {
        const LdsStencil<M, 1, NC, 1, fast_math<PREC>()> S{s_u, s_f, s_v, s_sr, s_H, t, &s_f[0][0]};
        double F[3];
        if (!euler_interface_flux<1, 0, PREC, PREC == 0>(S, LdsSpeeds{s_al}, A.gamma, A.W, F))
            err |= kErrNonphysical;
#pragma unroll
        for (int c = 0; c < 3; ++c) s_F[c][t] = F[c];
    }
    __syncthreads();
    double lam[3] = {0.0, 0.0, 0.0};
    if (t < TN && g0 + t < n) {
        const int64_t idx = off + g0 + t;
        const double dt = A.dt[b], dx = A.dx[b], rdx = A.rdx[b];
        double u0v[3];
        stage_u0<3>(A.stage, A.u0, A.total, idx, u0v);
        double un[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double L = -flux_quotient<FAST>(s_F[c][t + 1] - s_F[c][t], dx, rdx);
            const int64_t o = c * A.total + idx;
            un[c] = rk3_stage<FAST>(A.stage, A.uin[o], L, dt, u0v[c]);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) A.out[c * A.total + idx] = un[c];
        err |= euler_speeds<1, FAST>(un, A.gamma, lam);
    }
    if (err) atomicOr(&A.err[b], err);
    const int src[3] = {0, 1, 2}, dst[3] = {0, 1, 2};
    // lane moves (through the staged rows measured 0.7% slower in the fast mode)
    block_slot_max<3, 3>(lam, flat1_slot(A, A.wr, b), src, dst);
    if (g0 == 0 && t < kFlat1Speeds)
        __hip_atomic_store(&flat1_slot(A, A.zero, b)[t], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void reset_queue_kernel(int32_t *q)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *q = 0;
}

}  // namespace wt

namespace {

using namespace wt;

uint64_t mix(uint64_t h, uint64_t v)
{
    h ^= v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
    return h;
}

uint64_t bits(double d)
{
    uint64_t b;
    std::memcpy(&b, &d, sizeof b);
    return b;
}

void free_batch(wt_ctx *c)
{
    (void)hipFree(c->f1_state);
    (void)hipFree(c->f1_tab);
    c->f1_state = nullptr;
    c->f1_tab = nullptr;
    c->f1_state_cap = c->f1_tab_cap = 0;
    (void)hipFree(c->B1);
    (void)hipFree(c->B2);
    (void)hipFree(c->b_n);
    (void)hipFree(c->b_off);
    (void)hipFree(c->b_dx);
    (void)hipFree(c->b_rdx);
    (void)hipFree(c->b_bc);
    (void)hipFree(c->b_order);
    (void)hipFree(c->b_queue);
    c->B1 = c->B2 = nullptr;
    c->b_n = c->b_off = nullptr;
    c->b_dx = c->b_rdx = nullptr;
    c->b_bc = c->b_order = c->b_queue = nullptr;
    c->bcap = 0;
    c->b_cap = 0;
}

void free_batch2(wt_ctx *c)
{
    (void)hipFree(c->BD);
    (void)hipFree(c->b2_tab);
    (void)hipFree(c->b2_order);
    (void)hipFree(c->b2_queue);
    (void)hipFree(c->f2_state);
    (void)hipFree(c->f2_tab);
    c->BD = nullptr;
    c->b2_tab = nullptr;
    c->b2_order = c->b2_queue = nullptr;
    c->f2_state = nullptr;
    c->f2_tab = nullptr;
    c->bdcap = 0;
    c->b2_cap = 0;
    c->f2_state_cap = 0;
    c->f2_tab_cap = 0;
}

}  // namespace

namespace wt {

void release_batched(wt_ctx *c)
{
    if (c->b_graph) (void)hipGraphExecDestroy(c->b_graph);
    if (c->b2_graph) (void)hipGraphExecDestroy(c->b2_graph);
    if (c->b_capture) (void)hipStreamDestroy(c->b_capture);
    c->b_graph = nullptr;
    c->b2_graph = nullptr;
    c->b_capture = nullptr;
    free_batch(c);
    free_batch2(c);
}

}  // namespace wt

namespace {

constexpr int kBatchVariants1D = 3;   // 1D: persistent 256 / 128 threads, flat
constexpr int kBatchVariants2D = 5;   // 2D: persistent 4x63 / 8x31 x tiles, flat 8x31 / 4x63, packed
constexpr uint64_t kAnyBatch = ~0ull; // variant key of wenotheta_set_batched_tiles: every batch

// The variant of a batch: the tuned one for its signature, a forced one, else 0.
int batch_variant(int var, uint64_t key, uint64_t sig)
{
    return key == sig || key == kAnyBatch ? var : 0;
}

// Signature of a batch for the tuned-variant lookup: sizes, layout, precision.
uint64_t batch_signature(int ndim, int64_t nprob, const int64_t *n0, const int64_t *n1,
                         int64_t total, int precision)
{
    uint64_t h = mix(mix(mix((uint64_t)ndim, (uint64_t)nprob), (uint64_t)total), (uint64_t)precision);
    for (int64_t b = 0; b < nprob; ++b) {
        h = mix(h, (uint64_t)n0[b]);
        if (n1) h = mix(h, (uint64_t)n1[b]);
    }
    return h;
}

// Persistent grid: as many workgroups as are resident at once, at most one per problem.
template <class Kernel>
wt_status persistent_grid(wt_ctx *c, Kernel k, int threads, int64_t nprob, int64_t *grid)
{
    int per_cu = 0, ncu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, threads, 0) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess)
        return WT_ERR_DEVICE;
    *grid = std::min<int64_t>((int64_t)std::max(per_cu, 1) * std::max(ncu, 1), nprob);
    return WT_OK;
}

// ---- 1D batches ----

// Validate a 1D batch, upload its tables and size the workspace; fills A.
wt_status prepare_1d(wt_ctx *c, int64_t nprob, const int64_t *n, const int64_t *offset,
                     const double *lo, const double *hi, const int32_t *bc, const wt_params *P,
                     double *u, int64_t total, int64_t nsteps, hipStream_t s, BatchArgs *A, bool flat)
{
    if (!c || !P || !u || !n || !offset || !lo || !hi || !bc) return WT_ERR_ARG;
    if (nprob < 1 || nprob > (int64_t(1) << 30) || total < 6 || nsteps < 0) return WT_ERR_ARG;
    if (P->system != WT_EULER) return WT_ERR_UNSUPPORTED;
    if (P->precision != WT_FP64 && P->precision != WT_FP32_RECON && P->precision != WT_FP64_FAST)
        return WT_ERR_ARG;
    if (P->gravity[0] != 0.0 || P->gravity[1] != 0.0 || P->gravity[2] != 0.0) return WT_ERR_UNSUPPORTED;
    if (!(P->cfl > 0.0) || !(P->eps > 0.0) || !(P->alpha_R >= 0.0) || !(P->gamma > 1.0))
        return WT_ERR_ARG;
    // problems must be valid and pairwise disjoint inside [0, total)
    std::vector<int64_t> idx(nprob);
    std::iota(idx.begin(), idx.end(), 0);
    for (int64_t b = 0; b < nprob; ++b) {
        if (n[b] < 6 || offset[b] < 0 || offset[b] > total - n[b]) return WT_ERR_ARG;
        if (!(hi[b] > lo[b]) ||
            (bc[b] != WT_PERIODIC && bc[b] != WT_TRANSMISSIVE && bc[b] != WT_REFLECTIVE))
            return WT_ERR_ARG;
    }
    std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return offset[a] < offset[b]; });
    for (int64_t k = 1; k < nprob; ++k)
        if (offset[idx[k - 1]] + n[idx[k - 1]] > offset[idx[k]]) return WT_ERR_ARG;
    // work queue: largest problems first (longest-processing-time order)
    std::vector<int32_t> order(nprob);
    for (int64_t b = 0; b < nprob; ++b) order[b] = (int32_t)b;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return n[a] > n[b]; });
    std::vector<double> dx(nprob), rdx(nprob);
    for (int64_t b = 0; b < nprob; ++b) {
        dx[b] = (hi[b] - lo[b]) / (double)n[b];
        rdx[b] = 1.0 / dx[b];
    }
    std::vector<int32_t> bcv(bc, bc + nprob);

    if (hipSetDevice(c->device) != hipSuccess) return WT_ERR_DEVICE;
    // workspace (allocated on first use of a size)
    const size_t need = (size_t)total * 3;
    if (need > c->bcap || nprob > c->b_cap) {
        if (hipStreamSynchronize(s) != hipSuccess) return WT_ERR_DEVICE;
        // the stage buffers are shared with the 2D batches: both graphs go
        if (c->b_graph) (void)hipGraphExecDestroy(c->b_graph);
        if (c->b2_graph) (void)hipGraphExecDestroy(c->b2_graph);
        c->b_graph = nullptr;
        c->b2_graph = nullptr;
        free_batch(c);
        if (hipMalloc(&c->B1, need * sizeof(double)) != hipSuccess ||
            hipMalloc(&c->B2, need * sizeof(double)) != hipSuccess ||
            hipMalloc(&c->b_n, nprob * sizeof(int64_t)) != hipSuccess ||
            hipMalloc(&c->b_off, nprob * sizeof(int64_t)) != hipSuccess ||
            hipMalloc(&c->b_dx, nprob * sizeof(double)) != hipSuccess ||
            hipMalloc(&c->b_rdx, nprob * sizeof(double)) != hipSuccess ||
            hipMalloc(&c->b_bc, nprob * sizeof(int32_t)) != hipSuccess ||
            hipMalloc(&c->b_order, nprob * sizeof(int32_t)) != hipSuccess ||
            hipMalloc(&c->b_queue, sizeof(int32_t)) != hipSuccess) {
            free_batch(c);
            (void)hipGetLastError();
            return WT_ERR_NOMEM;
        }
        c->bcap = need;
        c->b_cap = nprob;
    }
    // problem tables (small host-to-device copies, ordered on the stream)
    if (hipMemcpyAsync(c->b_n, n, nprob * sizeof(int64_t), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(c->b_off, offset, nprob * sizeof(int64_t), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(c->b_dx, dx.data(), nprob * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(c->b_rdx, rdx.data(), nprob * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(c->b_bc, bcv.data(), nprob * sizeof(int32_t), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(c->b_order, order.data(), nprob * sizeof(int32_t), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return WT_ERR_DEVICE;

    *A = BatchArgs{};
    A->u = u;
    A->U1 = c->B1;
    A->U2 = c->B2;
    A->total = total;
    A->n = c->b_n;
    A->off = c->b_off;
    A->dx = c->b_dx;
    A->rdx = c->b_rdx;
    A->bc = c->b_bc;
    A->order = c->b_order;
    A->queue = c->b_queue;
    A->st = c->st;
    A->nprob = (int)nprob;
    A->nsteps = nsteps;
    A->gamma = P->gamma;
    A->W = WenoConst{P->eps, P->alpha_R, 1.0 / P->eps};
    A->cfl = P->cfl;
    if (!flat) return WT_OK;

    // flat form: the 255-point segments of all problems, problem by problem
    int64_t nft = 0;
    for (int64_t b = 0; b < nprob; ++b) nft += (n[b] + kThreads - 2) / (kThreads - 1);
    if (2 * nft > (int64_t(1) << 31)) return WT_ERR_ARG;
    std::vector<int32_t> ttab(2 * nft);
    for (int64_t b = 0, k = 0; b < nprob; ++b)
        for (int64_t j = 0, m = (n[b] + kThreads - 2) / (kThreads - 1); j < m; ++j, ++k) {
            ttab[k] = (int32_t)b;
            ttab[nft + k] = (int32_t)j;
        }
    const size_t state_bytes = (size_t)nprob * (3 * kFlat1Speeds * sizeof(unsigned long long) +
                                                2 * sizeof(double) + sizeof(int64_t) + sizeof(int32_t));
    if (nprob > c->f1_state_cap || 2 * nft > c->f1_tab_cap) {
        if (hipStreamSynchronize(s) != hipSuccess) return WT_ERR_DEVICE;
        if (c->b_graph) (void)hipGraphExecDestroy(c->b_graph);
        c->b_graph = nullptr;
        (void)hipFree(c->f1_state);
        (void)hipFree(c->f1_tab);
        c->f1_state = nullptr;
        c->f1_tab = nullptr;
        c->f1_state_cap = c->f1_tab_cap = 0;
        if (hipMalloc(&c->f1_state, state_bytes) != hipSuccess ||
            hipMalloc(&c->f1_tab, 2 * nft * sizeof(int32_t)) != hipSuccess) {
            (void)hipFree(c->f1_state);
            (void)hipFree(c->f1_tab);
            c->f1_state = nullptr;
            c->f1_tab = nullptr;
            (void)hipGetLastError();
            return WT_ERR_NOMEM;
        }
        c->f1_state_cap = nprob;
        c->f1_tab_cap = 2 * nft;
    }
    if (hipMemcpyAsync(c->f1_tab, ttab.data(), 2 * nft * sizeof(int32_t), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return WT_ERR_DEVICE;
    A->ft_prob = c->f1_tab;
    A->ft_local = c->f1_tab + nft;
    A->nft = nft;
    char *p = (char *)c->f1_state;
    A->f_spd = (unsigned long long *)p;
    p += (size_t)nprob * 3 * kFlat1Speeds * sizeof(unsigned long long);
    A->f_dt = (double *)p;
    p += (size_t)nprob * sizeof(double);
    A->f_time = (double *)p;
    p += (size_t)nprob * sizeof(double);
    A->f_first = (int64_t *)p;
    p += (size_t)nprob * sizeof(int64_t);
    A->f_err = (int32_t *)p;
    return WT_OK;
}

// The 1D flat form on stream s: initial speeds, nsteps x (time step, 3 passes), outputs.
wt_status enqueue_1d_flat(const BatchArgs &B, int precision, hipStream_t s)
{
    Flat1Args F{};
    F.total = B.total;
    F.n = B.n;
    F.off = B.off;
    F.dx = B.dx;
    F.rdx = B.rdx;
    F.bc = B.bc;
    F.tile_prob = B.ft_prob;
    F.tile_local = B.ft_local;
    F.ntiles = B.nft;
    F.tiles_per_xcd = (B.nft + kXcds - 1) / kXcds;
    F.spd = B.f_spd;
    F.dt = B.f_dt;
    F.time = B.f_time;
    F.err = B.f_err;
    F.first = B.f_first;
    F.nprob = B.nprob;
    F.nsteps = B.nsteps;
    F.gamma = B.gamma;
    F.cfl = B.cfl;
    F.W = B.W;
    F.t_out = B.t_out;
    F.status_out = B.status_out;
    F.steps_out = B.steps_out;
    F.st = B.st;
    const unsigned per_problem = (unsigned)((B.nprob + 255) / 256);
    const dim3 grid((unsigned)(F.tiles_per_xcd * kXcds)), block(kThreads);
    F.uin = B.u;
    hipLaunchKernelGGL(flat1_init_kernel, dim3((unsigned)B.nprob), dim3(kThreads), 0, s, F);
    for (int64_t step = 0; step < B.nsteps; ++step) {
        F.step = step;
        hipLaunchKernelGGL(flat1_dt_kernel, dim3(per_problem), dim3(256), 0, s, F);
        for (int stage = 1; stage <= 3; ++stage) {
            F.stage = stage;
            F.uin = stage == 1 ? B.u : (stage == 2 ? B.U1 : B.U2);
            F.out = stage == 1 ? B.U1 : (stage == 2 ? B.U2 : B.u);
            F.u0 = B.u;
            F.rd = stage - 1;
            F.wr = stage % 3;
            F.zero = (stage + 1) % 3;
            if (precision == WT_FP32_RECON) hipLaunchKernelGGL(flat1_pass_kernel<1>, grid, block, 0, s, F);
            else if (precision == WT_FP64_FAST) hipLaunchKernelGGL(flat1_pass_kernel<2>, grid, block, 0, s, F);
            else hipLaunchKernelGGL(flat1_pass_kernel<0>, grid, block, 0, s, F);
        }
    }
    hipLaunchKernelGGL(flat1_finish_kernel, dim3(per_problem), dim3(256), 0, s, F);
    return hipGetLastError() == hipSuccess ? WT_OK : WT_ERR_DEVICE;
}

// The 1D batch in variant v on s: the persistent kernel with workgroups of 256 (0)
// or 128 threads (1), or the flat form (2).
wt_status enqueue_1d(wt_ctx *c, const BatchArgs &A, int precision, int v, hipStream_t s)
{
    if (v == 2) return enqueue_1d_flat(A, precision, s);
    int64_t grid = 0;
    wt_status r;
    const int threads = v == 0 ? 256 : 128;
    if (precision == WT_FP32_RECON)
        r = v == 0 ? persistent_grid(c, batched_kernel<1, 256>, threads, A.nprob, &grid)
                   : persistent_grid(c, batched_kernel<1, 128>, threads, A.nprob, &grid);
    else if (precision == WT_FP64_FAST)
        r = v == 0 ? persistent_grid(c, batched_kernel<2, 256>, threads, A.nprob, &grid)
                   : persistent_grid(c, batched_kernel<2, 128>, threads, A.nprob, &grid);
    else
        r = v == 0 ? persistent_grid(c, batched_kernel<0, 256>, threads, A.nprob, &grid)
                   : persistent_grid(c, batched_kernel<0, 128>, threads, A.nprob, &grid);
    if (r != WT_OK) return r;
    hipLaunchKernelGGL(reset_queue_kernel, dim3(1), dim3(64), 0, s, A.queue);
    const dim3 g((unsigned)grid), b((unsigned)threads);
    if (precision == WT_FP32_RECON) {
        if (v == 0) hipLaunchKernelGGL((batched_kernel<1, 256>), g, b, 0, s, A);
        else hipLaunchKernelGGL((batched_kernel<1, 128>), g, b, 0, s, A);
    } else if (precision == WT_FP64_FAST) {
        if (v == 0) hipLaunchKernelGGL((batched_kernel<2, 256>), g, b, 0, s, A);
        else hipLaunchKernelGGL((batched_kernel<2, 128>), g, b, 0, s, A);
    } else {
        if (v == 0) hipLaunchKernelGGL((batched_kernel<0, 256>), g, b, 0, s, A);
        else hipLaunchKernelGGL((batched_kernel<0, 128>), g, b, 0, s, A);
    }
    return hipGetLastError() == hipSuccess ? WT_OK : WT_ERR_DEVICE;
}

// ---- 2D batches ----

// Tiles of a pass over lines of nd points (nl lines) in TX x TN tiles.
int64_t pass_tiles(int64_t nd, int64_t nl, int tx, int tn)
{
    return ((nl + tx - 1) / tx) * ((nd + tn - 1) / tn);
}

wt_status prepare_2d(wt_ctx *c, int64_t nprob, const int64_t *nx, const int64_t *ny,
                     const int64_t *offset, const double *lo, const double *hi, const int32_t *bc,
                     const wt_params *P, double *u, int64_t total, int64_t nsteps, hipStream_t s,
                     Batch2Args *A, bool flat)
{
    if (!c || !P || !u || !nx || !ny || !offset || !lo || !hi || !bc) return WT_ERR_ARG;
    if (nprob < 1 || nprob > (int64_t(1) << 30) || total < 36 || nsteps < 0) return WT_ERR_ARG;
    if (P->system != WT_EULER) return WT_ERR_UNSUPPORTED;
    if (P->precision != WT_FP64 && P->precision != WT_FP32_RECON && P->precision != WT_FP64_FAST)
        return WT_ERR_ARG;
    if (P->gravity[0] != 0.0 || P->gravity[1] != 0.0 || P->gravity[2] != 0.0) return WT_ERR_UNSUPPORTED;
    if (!(P->cfl > 0.0) || !(P->eps > 0.0) || !(P->alpha_R >= 0.0) || !(P->gamma > 1.0))
        return WT_ERR_ARG;
    // problems must be valid and pairwise disjoint inside [0, total)
    std::vector<Prob2> tab(nprob);
    std::vector<int64_t> cells(nprob);
    for (int64_t b = 0; b < nprob; ++b) {
        if (nx[b] < 6 || ny[b] < 6 || nx[b] > total || ny[b] > total / nx[b] || offset[b] < 0) return WT_ERR_ARG;
        // the packed chunks index a pass's interfaces of one problem in 32 bits
        if ((nx[b] + 1) * ny[b] > (int64_t(1) << 30) || (ny[b] + 1) * nx[b] > (int64_t(1) << 30))
            return WT_ERR_ARG;
        cells[b] = nx[b] * ny[b];
        if (offset[b] > total - cells[b]) return WT_ERR_ARG;
        for (int d = 0; d < 2; ++d) {
            const int32_t k = bc[2 * b + d];
            if (!(hi[2 * b + d] > lo[2 * b + d]) ||
                (k != WT_PERIODIC && k != WT_TRANSMISSIVE && k != WT_REFLECTIVE))
                return WT_ERR_ARG;
        }
        Prob2 &q = tab[b];
        q.nx = nx[b];
        q.ny = ny[b];
        q.off = offset[b];
        q.dx = (hi[2 * b] - lo[2 * b]) / (double)nx[b];
        q.rdx = 1.0 / q.dx;
        q.dy = (hi[2 * b + 1] - lo[2 * b + 1]) / (double)ny[b];
        q.rdy = 1.0 / q.dy;
        q.bcx = bc[2 * b];
        q.bcy = bc[2 * b + 1];
    }
    std::vector<int64_t> idx(nprob);
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return offset[a] < offset[b]; });
    for (int64_t k = 1; k < nprob; ++k)
        if (offset[idx[k - 1]] + cells[idx[k - 1]] > offset[idx[k]]) return WT_ERR_ARG;
    // work queue: largest problems first
    std::vector<int32_t> order(nprob);
    for (int64_t b = 0; b < nprob; ++b) order[b] = (int32_t)b;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return cells[a] > cells[b]; });

    if (hipSetDevice(c->device) != hipSuccess) return WT_ERR_DEVICE;
    // workspace: stage buffers shared with the 1D batches, then D and the tables
    const size_t need = (size_t)total * 4;
    if (need > c->bcap) {
        if (hipStreamSynchronize(s) != hipSuccess) return WT_ERR_DEVICE;
        if (c->b_graph) (void)hipGraphExecDestroy(c->b_graph);
        if (c->b2_graph) (void)hipGraphExecDestroy(c->b2_graph);
        c->b_graph = nullptr;
        c->b2_graph = nullptr;
        (void)hipFree(c->B1);
        (void)hipFree(c->B2);
        c->B1 = c->B2 = nullptr;
        c->bcap = 0;
        if (hipMalloc(&c->B1, need * sizeof(double)) != hipSuccess ||
            hipMalloc(&c->B2, need * sizeof(double)) != hipSuccess) {
            (void)hipFree(c->B1);
            (void)hipFree(c->B2);
            c->B1 = c->B2 = nullptr;
            (void)hipGetLastError();
            return WT_ERR_NOMEM;
        }
        c->bcap = need;
    }
    if (need > c->bdcap || nprob > c->b2_cap) {
        if (hipStreamSynchronize(s) != hipSuccess) return WT_ERR_DEVICE;
        if (c->b2_graph) (void)hipGraphExecDestroy(c->b2_graph);
        c->b2_graph = nullptr;
        free_batch2(c);
        if (hipMalloc(&c->BD, need * sizeof(double)) != hipSuccess ||
            hipMalloc(&c->b2_tab, nprob * sizeof(Prob2)) != hipSuccess ||
            hipMalloc(&c->b2_order, nprob * sizeof(int32_t)) != hipSuccess ||
            hipMalloc(&c->b2_queue, sizeof(int32_t)) != hipSuccess) {
            free_batch2(c);
            (void)hipGetLastError();
            return WT_ERR_NOMEM;
        }
        c->bdcap = need;
        c->b2_cap = nprob;
    }
    if (hipMemcpyAsync(c->b2_tab, tab.data(), nprob * sizeof(Prob2), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(c->b2_order, order.data(), nprob * sizeof(int32_t), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return WT_ERR_DEVICE;

    *A = Batch2Args{};
    A->u = u;
    A->U1 = c->B1;
    A->U2 = c->B2;
    A->D = c->BD;
    A->total = total;
    A->prob = (const Prob2 *)c->b2_tab;
    A->order = c->b2_order;
    A->queue = c->b2_queue;
    A->st = c->st;
    A->nprob = (int)nprob;
    A->nsteps = nsteps;
    A->gamma = P->gamma;
    A->cfl = P->cfl;
    A->W = WenoConst{P->eps, P->alpha_R, 1.0 / P->eps};
    if (!flat) return WT_OK;

    // flat form: tile tables, problem by problem (x pass in 8 x 31 and in 4 x 63
    // tiles, y pass in 8 x 31), and the per-problem state
    int64_t ntx[2] = {0, 0}, nty = 0;
    for (int64_t b = 0; b < nprob; ++b) {
        ntx[0] += pass_tiles(nx[b], ny[b], 8, 31);
        ntx[1] += pass_tiles(nx[b], ny[b], 4, 63);
        nty += pass_tiles(ny[b], nx[b], 8, 31);
    }
    const int64_t entries = 2 * (ntx[0] + ntx[1] + nty);
    if (entries > (int64_t(1) << 31)) return WT_ERR_ARG;
    std::vector<int32_t> ttab(entries);
    int64_t pos = 0;
    auto list = [&](int64_t n, auto tiles_of) {   // (problem, local tile) pairs as two arrays
        int64_t k = 0;
        for (int64_t b = 0; b < nprob; ++b)
            for (int64_t j = 0, m = tiles_of(b); j < m; ++j, ++k) {
                ttab[pos + k] = (int32_t)b;
                ttab[pos + n + k] = (int32_t)j;
            }
        pos += 2 * n;
    };
    list(ntx[0], [&](int64_t b) { return pass_tiles(nx[b], ny[b], 8, 31); });
    list(ntx[1], [&](int64_t b) { return pass_tiles(nx[b], ny[b], 4, 63); });
    list(nty, [&](int64_t b) { return pass_tiles(ny[b], nx[b], 8, 31); });
    // packed chunks (wt_pack.hpp): x over groups of 8 rows, y over groups of 8 columns
    int64_t npk[2] = {0, 0};
    std::vector<int32_t> pk[2];
    for (int d = 0; d < 2; ++d) {
        std::vector<int32_t> pb, pq, pn;
        for (int64_t b = 0; b < nprob; ++b) {
            const int Wd = (int)(d == 0 ? nx[b] : ny[b]) + 1;
            const int nl = (int)((d == 0 ? ny[b] : nx[b]) + kPackLanes - 1) / kPackLanes;
            pack_chunks(Wd, nl, kPackQt, kPackRows,
                        [&](int q0, int nq) {
                            pb.push_back((int32_t)b);
                            pq.push_back(q0);
                            pn.push_back(nq);
                        });
        }
        npk[d] = (int64_t)pb.size();
        pk[d].reserve(3 * pb.size());
        pk[d].insert(pk[d].end(), pb.begin(), pb.end());
        pk[d].insert(pk[d].end(), pq.begin(), pq.end());
        pk[d].insert(pk[d].end(), pn.begin(), pn.end());
    }
    if (entries + 3 * (npk[0] + npk[1]) > (int64_t(1) << 31)) return WT_ERR_ARG;
    ttab.insert(ttab.end(), pk[0].begin(), pk[0].end());
    ttab.insert(ttab.end(), pk[1].begin(), pk[1].end());
    const int64_t all_entries = (int64_t)ttab.size();
    const size_t state_bytes = (size_t)nprob * (3 * kFlatSpeeds * sizeof(unsigned long long) +
                                                2 * sizeof(double) + sizeof(int32_t) + sizeof(int64_t));
    if (nprob > c->f2_state_cap || all_entries > c->f2_tab_cap) {
        if (hipStreamSynchronize(s) != hipSuccess) return WT_ERR_DEVICE;
        if (c->b2_graph) (void)hipGraphExecDestroy(c->b2_graph);
        c->b2_graph = nullptr;
        (void)hipFree(c->f2_state);
        (void)hipFree(c->f2_tab);
        c->f2_state = nullptr;
        c->f2_tab = nullptr;
        c->f2_state_cap = c->f2_tab_cap = 0;
        if (hipMalloc(&c->f2_state, state_bytes) != hipSuccess ||
            hipMalloc(&c->f2_tab, all_entries * sizeof(int32_t)) != hipSuccess) {
            (void)hipFree(c->f2_state);
            (void)hipFree(c->f2_tab);
            c->f2_state = nullptr;
            c->f2_tab = nullptr;
            (void)hipGetLastError();
            return WT_ERR_NOMEM;
        }
        c->f2_state_cap = nprob;
        c->f2_tab_cap = all_entries;
    }
    if (hipMemcpyAsync(c->f2_tab, ttab.data(), all_entries * sizeof(int32_t), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return WT_ERR_DEVICE;
    const int32_t *t0 = c->f2_tab;
    A->xt_prob[0] = t0;
    A->xt_local[0] = t0 + ntx[0];
    A->xt_prob[1] = t0 + 2 * ntx[0];
    A->xt_local[1] = t0 + 2 * ntx[0] + ntx[1];
    A->yt_prob = t0 + 2 * (ntx[0] + ntx[1]);
    A->yt_local = A->yt_prob + nty;
    A->ntx[0] = ntx[0];
    A->ntx[1] = ntx[1];
    A->nty = nty;
    const int32_t *pk0 = t0 + entries;
    for (int d = 0; d < 2; ++d) {
        A->pk_prob[d] = pk0;
        A->pk_q0[d] = pk0 + npk[d];
        A->pk_n[d] = pk0 + 2 * npk[d];
        A->npk[d] = npk[d];
        pk0 += 3 * npk[d];
    }
    char *p = (char *)c->f2_state;
    A->f_spd = (unsigned long long *)p;
    p += (size_t)nprob * 3 * kFlatSpeeds * sizeof(unsigned long long);
    A->f_dt = (double *)p;
    p += (size_t)nprob * sizeof(double);
    A->f_time = (double *)p;
    p += (size_t)nprob * sizeof(double);
    A->f_first = (int64_t *)p;
    p += (size_t)nprob * sizeof(int64_t);
    A->f_err = (int32_t *)p;
    return WT_OK;
}

// The flat form on stream s: initial speeds, nsteps x (time step, 3 x (x pass,
// y pass)), outputs.  xv: x tiles 8 x 31 (0) or 4 x 63 (1).
wt_status enqueue_2d_flat(const Batch2Args &B, int precision, int xv, hipStream_t s)
{
    Flat2Args F{};
    F.total = B.total;
    F.prob = B.prob;
    F.D = B.D;
    F.spd = B.f_spd;
    F.dt = B.f_dt;
    F.time = B.f_time;
    F.err = B.f_err;
    F.first = B.f_first;
    F.nprob = B.nprob;
    F.nsteps = B.nsteps;
    F.gamma = B.gamma;
    F.cfl = B.cfl;
    F.W = B.W;
    F.t_out = B.t_out;
    F.status_out = B.status_out;
    F.steps_out = B.steps_out;
    F.st = B.st;
    const unsigned per_problem = (unsigned)((B.nprob + 255) / 256);
    F.uin = B.u;
    hipLaunchKernelGGL(flat2_init_kernel, dim3((unsigned)B.nprob), dim3(kThreads), 0, s, F);
    auto pass = [&](int dir, const int32_t *tp, const int32_t *tl, int64_t n) {
        Flat2Args G = F;
        G.tile_prob = tp;
        G.tile_local = tl;
        G.ntiles = n;
        G.tiles_per_xcd = (n + kXcds - 1) / kXcds;
        const dim3 grid((unsigned)(G.tiles_per_xcd * kXcds)), block(kThreads);
        if (xv == 2) {              // packed chunks of both passes
            G.tile_count = B.pk_n[dir];
            if (dir == 0) {
                if (precision == WT_FP32_RECON) hipLaunchKernelGGL((flat2_packed_kernel<0, 1>), grid, block, 0, s, G);
                else if (precision == WT_FP64_FAST) hipLaunchKernelGGL((flat2_packed_kernel<0, 2>), grid, block, 0, s, G);
                else hipLaunchKernelGGL((flat2_packed_kernel<0, 0>), grid, block, 0, s, G);
            } else {
                if (precision == WT_FP32_RECON) hipLaunchKernelGGL((flat2_packed_kernel<1, 1>), grid, block, 0, s, G);
                else if (precision == WT_FP64_FAST) hipLaunchKernelGGL((flat2_packed_kernel<1, 2>), grid, block, 0, s, G);
                else hipLaunchKernelGGL((flat2_packed_kernel<1, 0>), grid, block, 0, s, G);
            }
        } else if (dir == 0) {
            if (precision == WT_FP32_RECON) {
                if (xv == 0) hipLaunchKernelGGL((flat2_pass_kernel<0, 8, 31, 1>), grid, block, 0, s, G);
                else hipLaunchKernelGGL((flat2_pass_kernel<0, 4, 63, 1>), grid, block, 0, s, G);
            } else if (precision == WT_FP64_FAST) {
                if (xv == 0) hipLaunchKernelGGL((flat2_pass_kernel<0, 8, 31, 2>), grid, block, 0, s, G);
                else hipLaunchKernelGGL((flat2_pass_kernel<0, 4, 63, 2>), grid, block, 0, s, G);
            } else {
                if (xv == 0) hipLaunchKernelGGL((flat2_pass_kernel<0, 8, 31, 0>), grid, block, 0, s, G);
                else hipLaunchKernelGGL((flat2_pass_kernel<0, 4, 63, 0>), grid, block, 0, s, G);
            }
        } else {
            if (precision == WT_FP32_RECON)
                hipLaunchKernelGGL((flat2_pass_kernel<1, 8, 31, 1>), grid, block, 0, s, G);
            else if (precision == WT_FP64_FAST)
                hipLaunchKernelGGL((flat2_pass_kernel<1, 8, 31, 2>), grid, block, 0, s, G);
            else
                hipLaunchKernelGGL((flat2_pass_kernel<1, 8, 31, 0>), grid, block, 0, s, G);
        }
    };
    for (int64_t step = 0; step < B.nsteps; ++step) {
        F.step = step;
        hipLaunchKernelGGL(flat2_dt_kernel, dim3(per_problem), dim3(256), 0, s, F);
        for (int stage = 1; stage <= 3; ++stage) {
            F.stage = stage;
            F.uin = stage == 1 ? B.u : (stage == 2 ? B.U1 : B.U2);
            F.out = stage == 1 ? B.U1 : (stage == 2 ? B.U2 : B.u);
            F.u0 = B.u;
            F.rd = stage - 1;
            F.wr = stage % 3;
            F.zero = (stage + 1) % 3;
            if (xv == 2) {
                pass(0, B.pk_prob[0], B.pk_q0[0], B.npk[0]);
                pass(1, B.pk_prob[1], B.pk_q0[1], B.npk[1]);
            } else {
                pass(0, B.xt_prob[xv], B.xt_local[xv], B.ntx[xv]);
                pass(1, B.yt_prob, B.yt_local, B.nty);
            }
        }
    }
    hipLaunchKernelGGL(flat2_finish_kernel, dim3(per_problem), dim3(256), 0, s, F);
    return hipGetLastError() == hipSuccess ? WT_OK : WT_ERR_DEVICE;
}

// The 2D batch in variant v on s: the persistent kernel with x tiles 4 x 63 (0)
// or 8 x 31 (1), or the flat form with x tiles 8 x 31 (2) or 4 x 63 (3), or with
// packed chunks in both passes (4).
wt_status enqueue_2d(wt_ctx *c, const Batch2Args &A, int precision, int v, hipStream_t s)
{
    if (v >= 2) return enqueue_2d_flat(A, precision, v - 2, s);
    int64_t grid = 0;
    wt_status r;
    if (precision == WT_FP32_RECON)
        r = v == 0 ? persistent_grid(c, batched2d_kernel<1, 0>, kThreads, A.nprob, &grid)
                   : persistent_grid(c, batched2d_kernel<1, 1>, kThreads, A.nprob, &grid);
    else if (precision == WT_FP64_FAST)
        r = v == 0 ? persistent_grid(c, batched2d_kernel<2, 0>, kThreads, A.nprob, &grid)
                   : persistent_grid(c, batched2d_kernel<2, 1>, kThreads, A.nprob, &grid);
    else
        r = v == 0 ? persistent_grid(c, batched2d_kernel<0, 0>, kThreads, A.nprob, &grid)
                   : persistent_grid(c, batched2d_kernel<0, 1>, kThreads, A.nprob, &grid);
    if (r != WT_OK) return r;
    hipLaunchKernelGGL(reset_queue_kernel, dim3(1), dim3(64), 0, s, A.queue);
    const dim3 g((unsigned)grid), b(kThreads);
    if (precision == WT_FP32_RECON) {
        if (v == 0) hipLaunchKernelGGL((batched2d_kernel<1, 0>), g, b, 0, s, A);
        else hipLaunchKernelGGL((batched2d_kernel<1, 1>), g, b, 0, s, A);
    } else if (precision == WT_FP64_FAST) {
        if (v == 0) hipLaunchKernelGGL((batched2d_kernel<2, 0>), g, b, 0, s, A);
        else hipLaunchKernelGGL((batched2d_kernel<2, 1>), g, b, 0, s, A);
    } else {
        if (v == 0) hipLaunchKernelGGL((batched2d_kernel<0, 0>), g, b, 0, s, A);
        else hipLaunchKernelGGL((batched2d_kernel<0, 1>), g, b, 0, s, A);
    }
    return hipGetLastError() == hipSuccess ? WT_OK : WT_ERR_DEVICE;
}

// Replay (capturing first if the arguments changed) the graph of an enqueue call.
template <class Enqueue>
wt_status run_graph(wt_ctx *c, hipGraphExec_t *exec, uint64_t *exec_key, uint64_t key,
                    hipStream_t s, Enqueue enqueue)
{
    if (!*exec || *exec_key != key) {
        if (*exec) (void)hipGraphExecDestroy(*exec);
        *exec = nullptr;
        if (!c->b_capture && hipStreamCreateWithFlags(&c->b_capture, hipStreamNonBlocking) != hipSuccess)
            return WT_ERR_DEVICE;
        hipGraph_t g = nullptr;
        if (hipStreamBeginCapture(c->b_capture, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return WT_ERR_DEVICE;
        const wt_status r = enqueue(c->b_capture);
        if (hipStreamEndCapture(c->b_capture, &g) != hipSuccess || r != WT_OK) {
            if (g) (void)hipGraphDestroy(g);
            return r != WT_OK ? r : WT_ERR_DEVICE;
        }
        const hipError_t e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            *exec = nullptr;
            return WT_ERR_DEVICE;
        }
        *exec_key = key;
    }
    return hipGraphLaunch(*exec, s) == hipSuccess ? WT_OK : WT_ERR_DEVICE;
}

uint64_t launch_key(const void *u, const void *t_out, const void *status_out, const void *steps_out,
                    const wt_ctx *c, int64_t nprob, int64_t total, int64_t nsteps, const wt_params *P,
                    int variant, uint64_t signature)
{
    uint64_t key = signature;
    for (uint64_t v : {(uint64_t)(uintptr_t)u, (uint64_t)(uintptr_t)t_out,
                       (uint64_t)(uintptr_t)status_out, (uint64_t)(uintptr_t)steps_out,
                       (uint64_t)(uintptr_t)c->B1, (uint64_t)(uintptr_t)c->B2,
                       (uint64_t)(uintptr_t)c->BD, (uint64_t)(uintptr_t)c->f2_state,
                       (uint64_t)(uintptr_t)c->f2_tab, (uint64_t)(uintptr_t)c->f1_state,
                       (uint64_t)(uintptr_t)c->f1_tab, (uint64_t)nprob, (uint64_t)total, (uint64_t)nsteps,
                       (uint64_t)P->precision, bits(P->gamma), bits(P->eps), bits(P->alpha_R),
                       bits(P->cfl), (uint64_t)variant})
        key = mix(key, v);
    return key;
}

// Time each tile variant on a scratch copy of the batch (probe_steps steps, 3 rounds
// interleaved, best launch kept); the default variant stays unless another is more
// than 2% faster.  prepare fills the kernel arguments for a state pointer.
template <class Args, class Prepare, class Enqueue>
wt_status tune_variants(wt_ctx *c, const double *u, size_t state_doubles, int64_t nprob,
                        int precision, int nvar, hipStream_t s, Prepare prepare, Enqueue enqueue,
                        int *best)
{
    double *scratch = nullptr;
    int32_t *status = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    wt_status r = WT_OK;
    float ms[kBatchVariants2D];
    for (int v = 0; v < nvar; ++v) ms[v] = 3.0e38f;
    if (hipMalloc(&scratch, state_doubles * sizeof(double)) != hipSuccess ||
        hipMalloc(&status, nprob * sizeof(int32_t)) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        r = WT_ERR_NOMEM;
    } else {
        Args A{};
        r = prepare(scratch, &A);
        A.status_out = status;          // non-physical problems are reported here, not in the context
        for (int round = 0; round < 3 && r == WT_OK; ++round)
            for (int v = 0; v < nvar && r == WT_OK; ++v) {
                if (hipMemcpyAsync(scratch, u, state_doubles * sizeof(double), hipMemcpyDeviceToDevice, s) !=
                        hipSuccess ||
                    hipEventRecord(e0, s) != hipSuccess) {
                    r = WT_ERR_DEVICE;
                    break;
                }
                r = enqueue(A, precision, v, s);
                float t = 0.0f;
                if (r == WT_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                   hipEventElapsedTime(&t, e0, e1) != hipSuccess))
                    r = WT_ERR_DEVICE;
                if (r == WT_OK && t < ms[v]) ms[v] = t;
            }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(scratch);
    (void)hipFree(status);
    if (r != WT_OK) {
        (void)hipGetLastError();
        return r;
    }
    int v_best = 0;
    for (int v = 1; v < nvar; ++v)
        if (ms[v] < 0.98f * ms[v_best]) v_best = v;
    *best = v_best;
    return WT_OK;
}

}  // namespace

extern "C" wt_status wenotheta_solve_batched(wt_ctx *c, int64_t nprob, const int64_t *n,
                                             const int64_t *offset, const double *lo,
                                             const double *hi, const int32_t *bc,
                                             const wt_params *P, double *u, int64_t total,
                                             int64_t nsteps, double *t_out, int32_t *status_out,
                                             int64_t *steps_out, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (!c || !P || !n) return WT_ERR_ARG;
    const uint64_t sig = batch_signature(1, nprob, n, nullptr, total, P->precision);
    const int v = batch_variant(c->b_var, c->b_var_key, sig);
    BatchArgs A;
    wt_status r = prepare_1d(c, nprob, n, offset, lo, hi, bc, P, u, total, nsteps, s, &A, v == 2);
    if (r != WT_OK) return r;
    A.t_out = t_out;
    A.status_out = status_out;
    A.steps_out = steps_out;
    const int prec = P->precision;
    return run_graph(c, &c->b_graph, &c->b_key,
                     launch_key(u, t_out, status_out, steps_out, c, nprob, total, nsteps, P, v, sig), s,
                     [&](hipStream_t cs) { return enqueue_1d(c, A, prec, v, cs); });
}

extern "C" wt_status wenotheta_solve_batched_2d(wt_ctx *c, int64_t nprob, const int64_t *nx,
                                                const int64_t *ny, const int64_t *offset,
                                                const double *lo, const double *hi,
                                                const int32_t *bc, const wt_params *P, double *u,
                                                int64_t total, int64_t nsteps, double *t_out,
                                                int32_t *status_out, int64_t *steps_out, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (!c || !P || !nx || !ny) return WT_ERR_ARG;
    const uint64_t sig = batch_signature(2, nprob, nx, ny, total, P->precision);
    const int v = batch_variant(c->b2_var, c->b2_var_key, sig);
    Batch2Args A;
    wt_status r = prepare_2d(c, nprob, nx, ny, offset, lo, hi, bc, P, u, total, nsteps, s, &A, v >= 2);
    if (r != WT_OK) return r;
    A.t_out = t_out;
    A.status_out = status_out;
    A.steps_out = steps_out;
    const int prec = P->precision;
    return run_graph(c, &c->b2_graph, &c->b2_key,
                     launch_key(u, t_out, status_out, steps_out, c, nprob, total, nsteps, P, v, sig), s,
                     [&](hipStream_t cs) { return enqueue_2d(c, A, prec, v, cs); });
}

extern "C" wt_status wenotheta_tune_batched(wt_ctx *c, int64_t nprob, const int64_t *n,
                                            const int64_t *offset, const double *lo,
                                            const double *hi, const int32_t *bc,
                                            const wt_params *P, const double *u, int64_t total,
                                            int64_t probe_steps, int32_t *variant_out, void *stream)
{
    if (!c || !P || !u || probe_steps < 1) return WT_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    int best = 0;
    const wt_status r = tune_variants<BatchArgs>(
        c, u, (size_t)total * 3, nprob, P->precision, kBatchVariants1D, s,
        [&](double *scratch, BatchArgs *A) {
            return prepare_1d(c, nprob, n, offset, lo, hi, bc, P, scratch, total, probe_steps, s, A, true);
        },
        [&](const BatchArgs &A, int prec, int v, hipStream_t cs) { return enqueue_1d(c, A, prec, v, cs); },
        &best);
    if (r != WT_OK) return r;
    c->b_var = best;
    c->b_var_key = batch_signature(1, nprob, n, nullptr, total, P->precision);
    if (variant_out) *variant_out = best;
    return WT_OK;
}

extern "C" wt_status wenotheta_tune_batched_2d(wt_ctx *c, int64_t nprob, const int64_t *nx,
                                               const int64_t *ny, const int64_t *offset,
                                               const double *lo, const double *hi,
                                               const int32_t *bc, const wt_params *P,
                                               const double *u, int64_t total, int64_t probe_steps,
                                               int32_t *variant_out, void *stream)
{
    if (!c || !P || !u || probe_steps < 1) return WT_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    int best = 0;
    const wt_status r = tune_variants<Batch2Args>(
        c, u, (size_t)total * 4, nprob, P->precision, kBatchVariants2D, s,
        [&](double *scratch, Batch2Args *A) {
            return prepare_2d(c, nprob, nx, ny, offset, lo, hi, bc, P, scratch, total, probe_steps, s, A,
                              true);
        },
        [&](const Batch2Args &A, int prec, int v, hipStream_t cs) { return enqueue_2d(c, A, prec, v, cs); },
        &best);
    if (r != WT_OK) return r;
    c->b2_var = best;
    c->b2_var_key = batch_signature(2, nprob, nx, ny, total, P->precision);
    if (variant_out) *variant_out = best;
    return WT_OK;
}

extern "C" wt_status wenotheta_set_batched_tiles(wt_ctx *c, int32_t ndim, int32_t variant)
{
    if (!c || (ndim != 1 && ndim != 2) || variant < 0 ||
        variant >= (ndim == 1 ? kBatchVariants1D : kBatchVariants2D))
        return WT_ERR_ARG;
    if (ndim == 1) {
        c->b_var = variant;
        c->b_var_key = kAnyBatch;
    } else {
        c->b2_var = variant;
        c->b2_var_key = kAnyBatch;
    }
    return WT_OK;
}
