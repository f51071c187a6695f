// MI355X (gfx950) implementation of the WENO-theta C ABI declared in
// include/wenotheta.h.
//
// Structure of one Runge-Kutta stage on an ndim-dimensional grid:
//   * one "sweep" kernel per direction.  A block owns a tile of TX columns x
//     TN points along the sweep direction; it stages the tile plus a 3-point
//     halo on both sides (the stencil S^6 of the interfaces it owns) in LDS,
//     converting each point once to the quantities the fluxes need, then one
//     thread per interface computes the characteristic-wise WENO-theta flux
//     (Roe basis, projection, Lax-Friedrichs split, two reconstructions per
//     field, back-projection), and the cells take flux differences;
//   * all sweeps but the last write / accumulate the divergence D; the last
//     one forms L = -(D_x + D_y + D_z), applies the stage of the TVD
//     Runge-Kutta scheme and, in an epilogue, reduces the Lax-Friedrichs
//     speeds of the new state for the next stage (wave shuffles, then one
//     atomic max per block and value, skipped when it cannot raise the value).
//
// Global quantities (Lax-Friedrichs speeds, dt, t, error flags) live in a
// small device struct of the context, so a whole solve runs without host
// round trips between steps.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>

#include "wenotheta.h"
#include "wt_flux.hpp"

#include "wt_device.hpp"

namespace wt {

enum : int { MODE_FIRST = 0, MODE_MID = 1, MODE_LAST_RHS = 2, MODE_LAST_STAGE = 3 };

struct SweepArgs {
    const double *uin;     // state whose fluxes are taken
    const double *u0;      // state at the start of the step (stages 2, 3)
    double *out;           // L (rhs) or the next stage state
    double *D;             // divergence accumulator (ndim > 1)
    const double *fgiven;  // caller flux point values (1D scalar rhs) or null
    DevState *st;
    int64_t n[3];
    int64_t ncell;
    double dx;             // spacing along the sweep
    double rdx;            // 1 / dx rounded to nearest (host-computed)
    double a;              // linear advection speed
    double gamma;
    WenoConst W;
    int bc;                // boundary condition along the sweep
    int slot_rd, slot_wr, slot_zero;
    int stage;             // 1..3 (MODE_LAST_STAGE)
    int check_done;
    int64_t tiles;         // y/z sweeps: tiles of the grid, and tiles per XCD
    int64_t tiles_per_xcd;
    double grav[3];        // gravitational acceleration along -x_d (Euler)
    int has_grav;          // any grav[d] != 0: the source is added to L
    int walls;             // a wall on the sweep's dimension: acoustic speeds paired
    // WT_SIDES: the lower and upper ends' sides, and the coordinate origin and
    // spacing of the axis their splits run along ((DIR + 1) mod ndim)
    wt_side side[2];
    double tlo, tdx;
};

// Time of the state a sweep differentiates: the context's time for a
// right-hand side (stage 0), t^n, t^n + dt and t^n + dt/2 for the stages of a
// step (the abscissae of the 3-stage scheme).
__device__ __forceinline__ double stage_time(const DevState *st, int stage)
{
    if (stage == 2) return st->tn + st->dt;
    if (stage == 3) return st->tn + 0.5 * st->dt;
    return stage == 1 ? st->tn : st->t;
}

// Ghost point gi (< 0 or >= nd) of a grid line of a WT_SIDES dimension (Sec.
// 4.3, TEST 9): the side of that end is split along the next axis; the
// line's coordinate there, lo + (jt + 1/2) dx, below the split point at the
// stage's time selects part 0.  A given state fills the point; a wall part is
// the mirror image with the normal momentum negated; otherwise zero gradient.
template <int NDIM, int DIR, int M>
__device__ __forceinline__ void side_point(const SweepArgs &A, const DevState *st, int64_t gi,
                                           int64_t nd, int64_t at, int64_t sstride, int64_t jt,
                                           double *uc)
{
    const wt_side &S = A.side[gi < 0 ? 0 : 1];
    int part = 0;
    if constexpr (NDIM > 1) {
        const double x = A.tlo + ((double)jt + 0.5) * A.tdx;
        part = x < S.split0 + S.split_speed * stage_time(st, A.stage) ? 0 : 1;
    }
    const int kind = S.kind[part];
    if (kind == WT_SIDE_STATE) {
#pragma unroll
        for (int c = 0; c < M; ++c) uc[c] = S.state[part][c];
        return;
    }
    const int rule = kind == WT_SIDE_REFLECTIVE ? WT_REFLECTIVE : WT_TRANSMISSIVE;
    const int64_t idx = at + map_index(gi, nd, rule) * sstride;
#pragma unroll
    for (int c = 0; c < M; ++c) uc[c] = A.uin[c * A.ncell + idx];
    if (reflected(gi, nd, rule)) uc[1 + DIR] = -uc[1 + DIR];
}


// ---------------------------------------------------------------------------
// Lax-Friedrichs speeds of a state (grid-stride reduction into one slot)
// ---------------------------------------------------------------------------
template <int SYS, int NDIM>
__global__ __launch_bounds__(kThreads) void alpha_kernel(const double *u, int64_t ncell, double a,
                                                         double gamma, DevState *st, int slot)
{
    constexpr int NV = SpeedLayout<SYS, NDIM>::NV;
    double v[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = 0.0;
    int err = 0;
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < ncell;
         i += (int64_t)gridDim.x * kThreads) {
        if constexpr (SYS == SYS_EULER) {
            double uc[NDIM + 2], lam[3 * NDIM];
#pragma unroll
            for (int c = 0; c < NDIM + 2; ++c) uc[c] = u[c * ncell + i];
            err |= euler_speeds<NDIM>(uc, gamma, lam);
#pragma unroll
            for (int k = 0; k < NV; ++k) v[k] = lam[k] > v[k] ? lam[k] : v[k];
        } else {
            const double x = u[i];
            if (!__builtin_isfinite(x)) err |= kErrNonfinite;
            const double sp = SYS == SYS_LINEAR ? __builtin_fabs(a) : __builtin_fabs(x);
            v[0] = sp > v[0] ? sp : v[0];
        }
    }
    if (err) atomicOr(&st->err, err);
    constexpr int NS = SpeedLayout<SYS, NDIM>::NS;
    int src[NS], idx[NS];
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        src[j] = SpeedLayout<SYS, NDIM>::value_of_slot(j);
        idx[j] = SpeedLayout<SYS, NDIM>::slot_index(j);
    }
    block_slot_max<NV, NS>(v, st->alpha[slot], src, idx);
}

// Set slot `slot` to the given values (or zero) and zero slot `zero_slot`.
struct SlotValues {
    double v[kSlotLen];
};

__global__ void set_slots_kernel(DevState *st, int slot, SlotValues vals, int zero_slot)
{
    const int k = threadIdx.x;
    if (k < kSlotLen) {
        st->alpha[slot][k] = double_to_bits(vals.v[k]);
        if (zero_slot >= 0) st->alpha[zero_slot][k] = 0ull;
    }
}

// ---------------------------------------------------------------------------
// Step bookkeeping: dt from the speeds of the step's initial state
// ---------------------------------------------------------------------------
struct StepArgs {
    DevState *st;
    int slot;            // speeds of u^n
    int ndim;
    int euler;
    double dx[3];
    double cfl;
    double dt_fixed;     // > 0: use it
    int clip;            // solve mode: clip to t_end, honour max_steps
};

__global__ void step_begin_kernel(StepArgs A)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    DevState *st = A.st;
    if (st->done) return;
    if (st->err) { st->done = 1; return; }
    if (A.clip && (!(st->t < st->t_end) || (st->max_steps >= 0 && st->steps >= st->max_steps))) {
        st->done = 1;
        return;
    }
    st->tn = st->t;
    double dt = A.dt_fixed;
    if (!(dt > 0.0)) {
        // dt = cfl / sum_d amax_d / dx_d, amax_d = max(|u_d| + c) = max(alpha_{d,0}, alpha_{d,2})
        double s = 0.0;
        for (int d = 0; d < A.ndim; ++d) {
            double am;
            if (A.euler) {
                const double l0 = bits_to_double(st->alpha[A.slot][d * 5 + 0]);
                const double l2 = bits_to_double(st->alpha[A.slot][d * 5 + 2]);
                am = l2 > l0 ? l2 : l0;
            } else {
                am = bits_to_double(st->alpha[A.slot][0]);
            }
            s = d == 0 ? div_rn(am, A.dx[0]) : s + div_rn(am, A.dx[d]);
        }
        dt = div_rn(A.cfl, s);
    }
    double t_next = st->t + dt;
    if (A.clip) {
        if (st->t + dt >= st->t_end - 1e-6 * dt) {
            dt = st->t_end - st->t;
            t_next = st->t_end;
        }
    }
    st->dt = dt;
    st->t = t_next;
    st->steps = st->steps + 1;
}

// set_t = 0 keeps the context's time (a single step starts from it).
__global__ void solve_init_kernel(DevState *st, double t0, double t_end, long long max_steps,
                                  int set_t)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (set_t) st->t = t0;
        st->t_end = t_end;
        st->steps = 0;
        st->max_steps = max_steps;
        st->done = 0;
    }
}

__global__ void set_time_kernel(DevState *st, double t)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) st->t = t;
}

// Undo the time advance of the last step begun (the tuner begins one to get a
// CFL dt but keeps no step).
__global__ void restore_time_kernel(DevState *st)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) st->t = st->tn;
}

__global__ void copy_dt_kernel(const DevState *st, double *dst)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = st->dt;
}

// ---------------------------------------------------------------------------
// Sweep kernel
// ---------------------------------------------------------------------------

// Minimum waves per SIMD the register allocation must allow (measured on the
// benchmark grids): 4 for the Euler sweeps, which then fit 128 VGPRs without
// spills in every precision mode.  At 5 waves (96 VGPRs) the fast FP64 and the
// FP32-weight 2D sweeps spill 36-52 bytes and ran 6% (3.02e9 against 3.21e9
// cell-updates/s) and 11% (2.81e9 against 3.15e9) slower on 2D Euler 4096^2.
template <int SYS, int NDIM, int PREC>
constexpr int sweep_min_waves()
{
    return SYS == WT_EULER ? 4 : 1;
}

// 1D Euler grids are short (65536 points fill only 257 one-interface-per-thread
// workgroups, one wave per SIMD): there each interface's characteristic fields go
// to separate threads, 85 interfaces per workgroup, which shortens each thread's
// dependency chain threefold (3% faster at 65536 points in FP64; the FP32 form,
// whose chains are shorter, ran 3% slower and keeps one interface per thread).
template <int SYS, int NDIM, int PREC>
constexpr bool split_fields()
{
    return SYS == WT_EULER && NDIM == 1 && PREC == WT_FP64;
}

template <int SYS, int NDIM, int DIR, int TX, int TN, int MODE, int PREC>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(sweep_min_waves<SYS, NDIM, PREC>())))
void sweep_kernel(SweepArgs A)
{
    constexpr int M = Ncomp<SYS, NDIM>::value;
    constexpr int NC = (TN + 6) * TX;           // staged points of the tile
    constexpr bool EULER = SYS == SYS_EULER;
    constexpr int NV = SpeedLayout<SYS, NDIM>::NV;
    // 1D Euler: the characteristic fields of an interface on separate threads
    constexpr bool SPLIT = split_fields<SYS, NDIM, PREC>();
    constexpr bool FAST = fast_math<PREC>();
    static_assert(SPLIT ? TX == 1 && M * (TN + 1) <= kThreads : TX * (TN + 1) == kThreads,
                  "one interface (or, split, one field of an interface) per thread");

    __shared__ double s_u[M][NC];
    __shared__ double s_f[M][NC];                 // normal flux (Euler) / flux values (scalar)
    __shared__ double s_v[EULER ? NDIM : 1][EULER ? NC : 1];
    __shared__ double s_sr[EULER ? NC : 1];
    __shared__ double s_H[EULER ? NC : 1];
    // FP32 forms and 3D: the interface fluxes take the place of the staged normal
    // fluxes, which nobody reads once every interface is done; the smaller tile lets
    // one more workgroup share a CU (5 instead of 4 for the FP32 2D sweeps, 4 instead
    // of 3 for 3D).  The FP64 1D and 2D sweeps are bound by registers at 4 waves.
    constexpr bool ALIAS_F = PREC != 0 || NDIM == 3;
    static_assert(!ALIAS_F || NC >= kThreads, "the flux rows fit in the staged rows");
    __shared__ double s_Fown[ALIAS_F ? 1 : M][ALIAS_F ? 1 : kThreads];
    double (*s_F)[kThreads];
    if constexpr (ALIAS_F) s_F = reinterpret_cast<double (*)[kThreads]>(&s_f[0][0]);
    else s_F = reinterpret_cast<double (*)[kThreads]>(&s_Fown[0][0]);
    __shared__ double s_h[SPLIT ? M : 1][SPLIT ? TN + 1 : 1];   // h_s per field and interface
    __shared__ double s_al[EULER ? M : 1];       // Lax-Friedrichs speed per field
    // Fast forms: each point's pressure, from which the normal flux is projected, in
    // the first row of the normal-flux buffer (no flux is staged; the interface
    // fluxes replace the row once every stencil has been read).
    constexpr bool PRESS = EULER && FAST && !SPLIT;
    static_assert(!PRESS || ALIAS_F, "the fast forms alias the interface fluxes too");
    double *s_p = &s_f[0][0];

    DevState *st = A.st;
    if (A.check_done && st->done) return;

    const int64_t nx = A.n[0], ny = A.n[1], nz = A.n[2];
    const int64_t nd = A.n[DIR];
    // sizes are non-negative: unsigned division by the tile constants
    const int64_t nseg = (int64_t)((uint64_t)(nd + TN - 1) / TN);
    const int64_t ngx = DIR == 0 ? 1 : (int64_t)((uint64_t)(nx + TX - 1) / TX);

    // block -> tile.  Workgroups are dealt to the 8 XCDs round-robin (block i to
    // XCD i mod 8), each with its own L2; the y/z tiles of neighbouring column
    // groups share cache lines (8 doubles are half a 128-byte line) and those of
    // neighbouring segments share halo rows.  So XCD x takes the contiguous tile
    // range [x * per, (x + 1) * per) in order, per = ceil(tiles / 8); the grid is
    // rounded up to a multiple of 8 and surplus blocks leave at once.
    int64_t b = blockIdx.x;
    if constexpr (DIR != 0) {
        const int64_t per = A.tiles_per_xcd;
        b = (b % kXcds) * per + b / kXcds;
        if (b >= A.tiles) return;
    }
    // tile -> (x0, seg, base): base is the offset of sweep index 0 of column x0
    // x-sweeps: TX rows (row = y + z * ny) from row0, each a segment of TN points;
    // y/z-sweeps: TX columns from x0.
    // The launch has fewer than 2^31 tiles (checked by the host), so the tile index
    // and every factor of the tile count fit 32 bits: the decode divides in 32-bit
    // unsigned arithmetic, which costs a few instructions where a 64-bit division
    // takes a long scalar sequence and a dozen vector ones.
    int64_t seg, x0 = 0, row0 = 0, base;
    int64_t sstride;
    int64_t tline = 0;                           // line index along the split axis (WT_SIDES)
    const int64_t nrows = ny * nz;
    const uint32_t ub = (uint32_t)b, useg = (uint32_t)nseg;
    if constexpr (DIR == 0) {
        const uint32_t q = ub / useg;
        seg = ub - q * useg;
        row0 = (int64_t)q * TX;
        base = row0 * nx;
        sstride = 1;
    } else {
        const uint32_t ugx = (uint32_t)ngx;
        const uint32_t r = ub / ugx;
        const int64_t gx = ub - r * ugx;
        const uint32_t q = r / useg;
        seg = r - q * useg;
        x0 = gx * TX;
        sstride = DIR == 1 ? nx : nx * ny;
        if constexpr (DIR == 1) {
            base = (int64_t)q * nx * ny + x0;   // q = z
            tline = q;
        } else {
            base = (int64_t)q * nx + x0;        // q = y
        }
    }
    const int64_t g0 = seg * TN;                 // first owned point along the sweep
    const int64_t ncell = A.ncell;

    // ---- stage the tile (owned points + 3-point halos) and the fields' speeds ----
    if constexpr (EULER) {
        if (threadIdx.x < M)
            s_al[threadIdx.x] = SlotSpeeds{st->alpha[A.slot_rd], DIR, A.walls != 0}(threadIdx.x);
    }
    int err = 0;
    // A block's waves stage at a raised issue priority, so that a newly started block
    // issues its loads ahead of the interface arithmetic of the CU's other blocks.
    constexpr bool PRIO_STAGING = EULER && NDIM >= 2;
    if constexpr (PRIO_STAGING) __builtin_amdgcn_s_setprio(2);
    // Point i of the tile (i < NC): its LDS entry li = r * TX + cx for point r along the
    // sweep of lane cx (x-tiles of several rows are read row by row: consecutive threads,
    // consecutive x), its index gi along the sweep and its line's offset xo from base.
    auto tile_point = [&](int i, int &li, int64_t &gi, int64_t &xo) {
        int r, cx;
        if constexpr (DIR == 0 && TX > 1) {
            cx = i / (TN + 6);
            r = i - cx * (TN + 6);
        } else {
            r = i / TX;
            cx = i % TX;
        }
        li = r * TX + cx;
        gi = g0 - 3 + r;
        if constexpr (DIR != 0) xo = x0 + cx < nx ? cx : nx - 1 - x0;
        else xo = (row0 + cx < nrows ? cx : nrows - 1 - row0) * nx;
    };
    if constexpr (EULER) {
        // The first and middle sweeps of a stage load every point a thread stages before
        // converting any, so a thread with two points waits for HBM once, not once per
        // point (the block's barrier waits for its slowest wave).  The stage-finishing
        // sweeps keep the loop: unrolled, the 2D one needs 98 VGPRs and loses its fifth
        // wave per SIMD.
        constexpr bool STAGE_LOADS_FIRST = MODE == MODE_FIRST || MODE == MODE_MID;
        constexpr int NIT = (NC + kThreads - 1) / kThreads;
        double ucs[NIT][M];
        int lis[NIT] = {};
        auto load_point = [&](int i, int it) {
            {
                int64_t gi, xo;
                tile_point(i, lis[it], gi, xo);
                double *uc = ucs[it];
                if (A.bc == WT_SIDES && (gi < 0 || gi >= nd)) {
                    int64_t jt;
                    if constexpr (DIR == 0) {
                        const int64_t row = row0 + xo / nx;
                        jt = NDIM == 3 ? row % ny : row;
                    } else {
                        jt = NDIM == 3 && DIR == 1 ? tline : x0 + xo;
                    }
                    side_point<NDIM, DIR, M>(A, st, gi, nd, base + xo, sstride, jt, uc);
                } else {
                    const int64_t idx = base + map_index(gi, nd, A.bc) * sstride + xo;
#pragma unroll
                    for (int c = 0; c < M; ++c) uc[c] = A.uin[c * ncell + idx];
                    if (reflected(gi, nd, A.bc)) uc[1 + DIR] = -uc[1 + DIR];
                }
            }
        };
        auto convert_point = [&](int it) {
            {
                const int li = lis[it];
                const double *uc = ucs[it];
                double vel[NDIM], p, H;
                const bool ok = euler_cell<NDIM, FAST>(uc, A.gamma, vel, p, H);
                if (!ok) {
                    bool fin = true;
#pragma unroll
                    for (int c = 0; c < M; ++c) fin = fin && __builtin_isfinite(uc[c]);
                    err |= fin ? kErrNonphysical : kErrNonfinite;
                }
#pragma unroll
                for (int c = 0; c < M; ++c) s_u[c][li] = uc[c];
                if constexpr (PRESS) {
                    s_p[li] = p;
                } else {
                    double fn[M];
                    euler_normal_flux<NDIM, DIR>(uc, vel, p, fn);
#pragma unroll
                    for (int c = 0; c < M; ++c) s_f[c][li] = fn[c];
                }
#pragma unroll
                for (int k = 0; k < NDIM; ++k) s_v[k][li] = vel[k];
                s_sr[li] = FAST ? sqrt_fast(uc[0]) : sqrt_rn(uc[0]);
                s_H[li] = H;
            }
        };
        if constexpr (STAGE_LOADS_FIRST) {
#pragma unroll
            for (int it = 0; it < NIT; ++it)
                if (threadIdx.x + it * kThreads < NC) load_point(threadIdx.x + it * kThreads, it);
#pragma unroll
            for (int it = 0; it < NIT; ++it)
                if (threadIdx.x + it * kThreads < NC) convert_point(it);
        } else {
            for (int i = threadIdx.x; i < NC; i += kThreads) {
                load_point(i, 0);
                convert_point(0);
            }
        }
    } else {
        for (int i = threadIdx.x; i < NC; i += kThreads) {
            int li;
            int64_t gi, xo;
            tile_point(i, li, gi, xo);
            const int64_t idx = base + map_index(gi, nd, A.bc) * sstride + xo;
            const double x = A.uin[idx];
            double f;
            if (A.fgiven) f = A.fgiven[idx];
            else if constexpr (SYS == SYS_LINEAR) f = A.a * x;
            else f = 0.5 * x * x;
            if (!__builtin_isfinite(x) || !__builtin_isfinite(f)) err |= kErrNonfinite;
            s_u[0][li] = x;
            s_f[0][li] = f;
        }
    }
    if constexpr (PRIO_STAGING) __builtin_amdgcn_s_setprio(0);
    if (err) atomicOr(&st->err, err);
    __syncthreads();

    // The cell a thread updates after the interfaces (t < TN * TX), and its inputs that
    // do not depend on the fluxes -- D of the earlier sweeps and u^n -- loaded before
    // the barriers that close the interface phase, so that they are in flight while
    // the block's last interfaces finish.
    // (The first sweep of a stage reads neither and locates its cell afterwards.)
    auto locate_cell = [&](int64_t &idx) -> bool {
        const int t = threadIdx.x, it = t / TX, cx = t % TX;
        idx = base + (g0 + it) * sstride + (DIR == 0 ? cx * nx : cx);
        return t < TN * TX && (DIR == 0 ? row0 + cx < nrows : x0 + cx < nx) && g0 + it < nd;
    };
    constexpr bool PRE_D = NDIM > 1 && MODE != MODE_FIRST;
    constexpr bool PREFETCH = PRE_D || MODE == MODE_LAST_STAGE;
    bool pre_cell = false;
    int64_t pre_idx = 0;
    double preD[M], u0v[M];
    auto prefetch_cell = [&]() {
        if constexpr (PREFETCH) {
            pre_cell = locate_cell(pre_idx);
            if (pre_cell) {
                if constexpr (PRE_D) {
#pragma unroll
                    for (int c = 0; c < M; ++c) preD[c] = A.D[c * ncell + pre_idx];
                }
                if constexpr (MODE == MODE_LAST_STAGE) stage_u0<M>(A.stage, A.u0, ncell, pre_idx, u0v);
            }
        }
    };

    // ---- 1D Euler: one characteristic field of an interface per thread ----
    if constexpr (SPLIT) {
        const int t = threadIdx.x;
        const int it = t / M, f = t - it * M;   // interface between points it-1 and it; field
        const bool valid = t < M * (TN + 1) && g0 + it <= nd;
        const LdsStencil<M, NDIM, NC, 1> S{s_u, s_f, s_v, s_sr, s_H, it};
        RoeBasis<NDIM> B{};
        if (valid) {
            B = interface_basis<NDIM, DIR, FAST>(S, A.gamma);
            const LdsSpeeds al{s_al};
            s_h[f][it] = euler_field_flux<NDIM, DIR, PREC, fresh_rows<NDIM, PREC>()>(S, B, f, al, A.W);
            if (f == 0 && !B.ok) atomicOr(&st->err, kErrNonphysical);
        }
        prefetch_cell();
        __syncthreads();
        // back-projection by the field-0 thread, fields in the order of the
        // one-thread form (so the same sums)
        if (valid && f == 0) {
            double acc[M], F[M];
#pragma unroll
            for (int k = 0; k < M; ++k) {
                const int fs = field_order(k);
                backproject_field<NDIM, DIR, fresh_rows<NDIM, PREC>()>(B, fs, s_h[fs][it], acc);
            }
            store_interface_flux<NDIM, DIR>(acc, F);
#pragma unroll
            for (int q = 0; q < M; ++q) s_F[q][it] = F[q];
        }
    }
    // ---- one interface per thread: interface between points it-1 and it ----
    else {
        const int t = threadIdx.x;
        const int it = t / TX, cx = t % TX;
        const bool valid = (DIR == 0 ? row0 + cx < nrows : x0 + cx < nx) && g0 + it <= nd;
        double F[M];
        if (valid) {
            if constexpr (EULER) {
                const LdsStencil<M, NDIM, NC, TX, PRESS> S{s_u, s_f, s_v, s_sr, s_H, t, s_p};
                const LdsSpeeds al{s_al};
                if (!euler_interface_flux<NDIM, DIR, PREC>(S, al, A.gamma, A.W, F))
                    atomicOr(&st->err, kErrNonphysical);
            } else {
                const LdsScalarStencil<NC, TX> S{s_u[0], s_f[0], t};
                F[0] = scalar_interface_flux<PREC>(S, bits_to_double(st->alpha[A.slot_rd][0]), A.W);
            }
        }
        prefetch_cell();
        if constexpr (ALIAS_F) __syncthreads();     // every stencil read of s_f is done
        if (valid) {
#pragma unroll
            for (int q = 0; q < M; ++q) s_F[q][t] = F[q];
        }
    }
    __syncthreads();

    // ---- cells: flux differences, then the mode's update ----
    double spd[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) spd[k] = 0.0;
    int err2 = 0;
    {
        const int t = threadIdx.x;
        int64_t idx = pre_idx;
        bool cell = pre_cell;
        if constexpr (!PREFETCH) {
            if (t < TN * TX) {
                const int it = t / TX, cx = t % TX;
                const int64_t g = g0 + it;
                if ((DIR == 0 ? row0 + cx < nrows : x0 + cx < nx) && g < nd) {
                    idx = base + g * sstride + (DIR == 0 ? cx * nx : cx);
                    cell = true;
                }
            }
        }
        if (cell) {
            double Lc[M];
#pragma unroll
            for (int c = 0; c < M; ++c) {
                const double Dd = flux_quotient<FAST>(s_F[c][t + TX] - s_F[c][t], A.dx, A.rdx);
                const int64_t o = c * ncell + idx;
                if constexpr (MODE == MODE_FIRST) {
                    A.D[o] = Dd;
                } else if constexpr (MODE == MODE_MID) {
                    A.D[o] = preD[c] + Dd;
                } else {
                    if constexpr (NDIM == 1) Lc[c] = -Dd;
                    else Lc[c] = -(preD[c] + Dd);
                }
            }
            // The stage's input state of an owned cell is tile entry t + 3 TX (owned
            // points are never mirror images), read from LDS instead of HBM.
            if constexpr (EULER && (MODE == MODE_LAST_RHS || MODE == MODE_LAST_STAGE)) {
                // gravity source (Sec. 4.3, TEST 6) of the stage's input state
                if (A.has_grav) {
                    const double rho = s_u[0][t + 3 * TX];
                    double e = 0.0;
#pragma unroll
                    for (int d = 0; d < NDIM; ++d) {
                        const double md = s_u[1 + d][t + 3 * TX];
                        Lc[1 + d] = Lc[1 + d] + (-(A.grav[d] * rho));
                        e = d == 0 ? A.grav[0] * md : e + A.grav[d] * md;
                    }
                    Lc[NDIM + 1] = Lc[NDIM + 1] + (-e);
                }
            }
            if constexpr (MODE == MODE_LAST_RHS) {
#pragma unroll
                for (int c = 0; c < M; ++c) A.out[c * ncell + idx] = Lc[c];
            } else if constexpr (MODE == MODE_LAST_STAGE) {
                const double dt = st->dt;
                double un[M];
#pragma unroll
                for (int c = 0; c < M; ++c)
                    un[c] = rk3_stage<FAST>(A.stage, s_u[c][t + 3 * TX], Lc[c], dt, u0v[c]);
#pragma unroll
                for (int c = 0; c < M; ++c) A.out[c * ncell + idx] = un[c];
                // Lax-Friedrichs speeds of the new state
                if constexpr (EULER) {
                    double lam[3 * NDIM];
                    err2 |= euler_speeds<NDIM, FAST>(un, A.gamma, lam);
#pragma unroll
                    for (int k = 0; k < NV; ++k) spd[k] = lam[k];
                } else {
                    if (!__builtin_isfinite(un[0])) err2 |= kErrNonfinite;
                    spd[0] = SYS == SYS_LINEAR ? __builtin_fabs(A.a) : __builtin_fabs(un[0]);
                }
            }
        }
    }
    if constexpr (MODE == MODE_LAST_STAGE) {
        if (err2) atomicOr(&st->err, err2);
        constexpr int NS = SpeedLayout<SYS, NDIM>::NS;
        int src[NS], sidx[NS];
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            src[j] = SpeedLayout<SYS, NDIM>::value_of_slot(j);
            sidx[j] = SpeedLayout<SYS, NDIM>::slot_index(j);
        }
        // 2D/3D Euler: the speeds through the staged state and flux rows, free once
        // every cell is updated (fewer instructions than lane moves); 1D grids,
        // whose launches are latency-bound, keep the lane moves and one barrier.
        // speed rows kept in s_u (as many as fit, at most NV), the rest in s_f
        constexpr int KA = (M * NC) / kThreads < NV ? (M * NC) / kThreads : NV;
        if constexpr (EULER && NDIM >= 2) {
            static_assert((NV - KA) * kThreads + NV * 16 <= M * NC,
                          "the speed rows and their partials fit in the staged rows");
            block_slot_max_lds<NV, NS, kThreads, KA>(spd, st->alpha[A.slot_wr], src, sidx,
                                                     &s_u[0][0], &s_f[0][0]);
        } else {
            block_slot_max<NV, NS, kThreads, NDIM == 2>(spd, st->alpha[A.slot_wr], src, sidx);
        }
        if (blockIdx.x == 0 && threadIdx.x < kSlotLen)
            __hip_atomic_store(&st->alpha[A.slot_zero][threadIdx.x], 0ull, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ---------------------------------------------------------------------------
// Fused stage of the 2D Euler system
// ---------------------------------------------------------------------------
// One launch per Runge-Kutta stage (or RHS): a block owns a tile of kFX x kFY
// points and stages it once with 3-point halos in both directions (the corners,
// which no stencil reads, are skipped); the x interfaces, then their flux
// differences (kept in registers), then the y interfaces, and the stage update.
// No divergence array goes through HBM and the stage input is read once (plus
// halos), against two sweeps that write and read back D.  The interfaces use the
// sweeps' routine, so every flux is the same operations on the same values: the
// results are the sweeps' bit for bit.
//
// LDS per block: the staged points (state, velocities, p, sqrt(rho), H: 9 doubles
// each) and one buffer for the normal fluxes of the current direction, which the
// interface fluxes replace once every stencil has been read: 77 KB, two blocks of
// 512 threads per CU (4 waves per SIMD).
//
// Lanes and LDS banks: the tile is kFX = 31 points wide, so a row has 32 x
// interfaces and every group of 32 lanes takes one row, reading 32 consecutive LDS
// words; the y interfaces, the y normal fluxes and the owned points run 32 lanes per
// row as well (31 columns, the 32nd lane idle), on flux rows of 32 words.  No access
// of a half-wave then straddles two rows, which would meet in the same banks.
constexpr int kFX = 31, kFY = 15, kFThreads = 512;
constexpr int kFL = 32;                      // lanes per tile row in every phase
constexpr int kFW = kFX + 6, kFH = kFY + 6, kFNP = kFW * kFH;
constexpr int kFXF = kFY * kFW;              // x phase: normal fluxes of rows 3 .. kFY + 2
constexpr int kFYF = kFH * kFL;              // y phase: normal fluxes of columns 3 .. kFX + 2
constexpr int kFBuf = kFXF > kFYF ? kFXF : kFYF;
static_assert(kFX + 1 == kFL && kFL * (kFY + 1) <= kFThreads,
              "one interface per thread in each phase, one row per 32 lanes");
static_assert(kFL * (kFY + 1) <= kFBuf, "interface fluxes fit");

struct Stage2dArgs {
    const double *uin;     // state whose fluxes are taken
    const double *u0;      // state at the start of the step (stages 2, 3)
    double *out;           // L (rhs) or the next stage state
    DevState *st;
    int64_t n[2];
    int64_t ncell;
    double dx[2], rdx[2];
    double gamma;
    WenoConst W;
    int bc[2];
    int walls[2];
    int slot_rd, slot_wr, slot_zero;
    int stage;
    int check_done;
    int64_t ntx, tiles, tiles_per_xcd;
    double grav[2];
    int has_grav;
};

// Stencil of one interface on the fused tile: point k at staged index base + k step,
// its normal flux at fbase + k fstep of the flux buffer.
template <int STEP, int FSTEP>
struct TileStencil {
    const double (*u)[kFNP];
    const double (*fn)[kFBuf];
    const double (*vel)[kFNP];
    const double *sq, *hh;
    int base, fbase;
    const double *pp;                            // pressures of the staged points
    static constexpr bool kPressure = true;
    __device__ double U(int k, int c) const { return u[c][base + k * STEP]; }
    __device__ double f(int k, int c) const { return fn[c][fbase + k * FSTEP]; }
    __device__ double p(int k) const { return pp[base + k * STEP]; }
    __device__ double v(int k, int d) const { return vel[d][base + k * STEP]; }
    __device__ double sr(int k) const { return sq[base + k * STEP]; }
    __device__ double H(int k) const { return hh[base + k * STEP]; }
};

template <int MODE, int PREC>
__global__ __launch_bounds__(kFThreads) __attribute__((amdgpu_waves_per_eu(4)))
void stage2d_kernel(Stage2dArgs A)
{
    constexpr int M = 4;
    constexpr bool FAST = fast_math<PREC>();
    constexpr int NV = SpeedLayout<SYS_EULER, 2>::NV;
    __shared__ double s_u[M][kFNP];
    __shared__ double s_v[2][kFNP];
    __shared__ double s_p[kFNP];
    __shared__ double s_sr[kFNP];
    __shared__ double s_H[kFNP];
    __shared__ double s_f[M][kFBuf];             // normal fluxes, then interface fluxes
    __shared__ double s_al[2][M];                // Lax-Friedrichs speed per direction and field

    DevState *st = A.st;
    if (A.check_done && st->done) return;
    const int64_t nx = A.n[0], ny = A.n[1], ncell = A.ncell;
    // tiles dealt to the XCDs in contiguous ranges (see sweep_kernel)
    int64_t b = blockIdx.x;
    b = (b % kXcds) * A.tiles_per_xcd + b / kXcds;
    if (b >= A.tiles) return;
    // fewer than 2^31 tiles (checked by the host): 32-bit division
    const uint32_t ty = (uint32_t)b / (uint32_t)A.ntx;
    const int64_t x0 = ((uint32_t)b - ty * (uint32_t)A.ntx) * (int64_t)kFX;
    const int64_t y0 = (int64_t)ty * kFY;
    const int nxt = (int)(nx - x0 < kFX ? nx - x0 : kFX);   // owned points of the tile
    const int nyt = (int)(ny - y0 < kFY ? ny - y0 : kFY);
    const int t = threadIdx.x;

    // ---- stage the tile and its halos (ghost points through each direction's map)
    // and the fields' speeds
    if (t < 2 * M) {
        const int d = t / M;
        s_al[d][t - d * M] = SlotSpeeds{st->alpha[A.slot_rd], d, A.walls[d] != 0}(t - d * M);
    }
    int err = 0;
    for (int i = t; i < kFNP; i += kFThreads) {
        const int iy = i / kFW, ix = i - iy * kFW;
        if ((ix < 3 || ix >= kFX + 3) && (iy < 3 || iy >= kFY + 3)) continue;   // corner
        const int64_t gx = x0 - 3 + ix, gy = y0 - 3 + iy;
        const int64_t idx = map_index(gy, ny, A.bc[1]) * nx + map_index(gx, nx, A.bc[0]);
        double uc[M];
#pragma unroll
        for (int c = 0; c < M; ++c) uc[c] = A.uin[c * ncell + idx];
        if (reflected(gx, nx, A.bc[0])) uc[1] = -uc[1];
        if (reflected(gy, ny, A.bc[1])) uc[2] = -uc[2];
        double vel[2], p, H;
        if (!euler_cell<2, FAST>(uc, A.gamma, vel, p, H)) {
            bool fin = true;
#pragma unroll
            for (int c = 0; c < M; ++c) fin = fin && __builtin_isfinite(uc[c]);
            err |= fin ? kErrNonphysical : kErrNonfinite;
        }
#pragma unroll
        for (int c = 0; c < M; ++c) s_u[c][i] = uc[c];
        s_v[0][i] = vel[0];
        s_v[1][i] = vel[1];
        s_p[i] = p;
        s_sr[i] = FAST ? sqrt_fast(uc[0]) : sqrt_rn(uc[0]);
        s_H[i] = H;
    }
    if (err) atomicOr(&st->err, err);
    __syncthreads();

    // ---- x direction: normal fluxes of rows 3 .. kFY + 2, then one interface per thread
    // (the fast forms project the normal flux from the state and the pressure and
    // stage none)
    if constexpr (!FAST) {
        for (int i = t; i < kFXF; i += kFThreads) {
            const int li = i + 3 * kFW;
            double uc[M], vel[2], fn[M];
#pragma unroll
            for (int c = 0; c < M; ++c) uc[c] = s_u[c][li];
            vel[0] = s_v[0][li];
            vel[1] = s_v[1][li];
            euler_normal_flux<2, 0>(uc, vel, s_p[li], fn);
#pragma unroll
            for (int c = 0; c < M; ++c) s_f[c][i] = fn[c];
        }
        __syncthreads();
    }
    double F[M];
    {
        const int fi = t % kFL, j = t / kFL;     // face between points fi-1, fi of row j
        const bool valid = j < kFY && fi <= nxt && j < nyt;
        if (valid) {
            const TileStencil<1, 1> S{s_u, s_f, s_v, s_sr, s_H, (j + 3) * kFW + fi, j * kFW + fi, s_p};
            const LdsSpeeds al{s_al[0]};
            if (!euler_interface_flux<2, 0, PREC, true>(S, al, A.gamma, A.W, F))
                atomicOr(&st->err, kErrNonphysical);
        }
        __syncthreads();                         // every stencil read of s_f is done
        if (valid) {
#pragma unroll
            for (int c = 0; c < M; ++c) s_f[c][j * kFL + fi] = F[c];
        }
    }
    __syncthreads();
    // x flux differences of the owned points, kept for the end of the stage
    const int ci = t % kFL, cj = t / kFL;
    const bool own = cj < kFY && ci < kFX && ci < nxt && cj < nyt;
    double Dx[M];
    if (own) {
#pragma unroll
        for (int c = 0; c < M; ++c) {
            const double d = s_f[c][cj * kFL + ci + 1] - s_f[c][cj * kFL + ci];
            Dx[c] = flux_quotient<FAST>(d, A.dx[0], A.rdx[0]);
        }
    }
    __syncthreads();

    // ---- y direction: normal fluxes of columns 3 .. kFX + 2, one interface per thread
    if constexpr (!FAST) {
        for (int i = t; i < kFYF; i += kFThreads) {
            const int iy = i / kFL, cx = i - iy * kFL;
            if (cx >= kFX) continue;             // the idle 32nd lane of a row
            const int li = iy * kFW + cx + 3;
            double uc[M], vel[2], fn[M];
#pragma unroll
            for (int c = 0; c < M; ++c) uc[c] = s_u[c][li];
            vel[0] = s_v[0][li];
            vel[1] = s_v[1][li];
            euler_normal_flux<2, 1>(uc, vel, s_p[li], fn);
#pragma unroll
            for (int c = 0; c < M; ++c) s_f[c][i] = fn[c];
        }
        __syncthreads();
    }
    {
        const int i = t % kFL, fj = t / kFL;     // face between points fj-1, fj of column i
        const bool valid = fj <= kFY && i < kFX && i < nxt && fj <= nyt;
        if (valid) {
            const TileStencil<kFW, kFL> S{s_u, s_f, s_v, s_sr, s_H, fj * kFW + i + 3, fj * kFL + i, s_p};
            const LdsSpeeds al{s_al[1]};
            if (!euler_interface_flux<2, 1, PREC, true>(S, al, A.gamma, A.W, F))
                atomicOr(&st->err, kErrNonphysical);
        }
        __syncthreads();
        if (valid) {
#pragma unroll
            for (int c = 0; c < M; ++c) s_f[c][fj * kFL + i] = F[c];
        }
    }
    __syncthreads();

    // ---- owned points: L = -(D_x + D_y) (+ source), then the stage
    double spd[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) spd[k] = 0.0;
    int err2 = 0;
    if (own) {
        const int64_t idx = (y0 + cj) * nx + x0 + ci;
        const int li = (cj + 3) * kFW + ci + 3;
        double u0v[M];
        if constexpr (MODE == MODE_LAST_STAGE) stage_u0<M>(A.stage, A.u0, ncell, idx, u0v);
        double Lc[M];
#pragma unroll
        for (int c = 0; c < M; ++c) {
            const double d = s_f[c][(cj + 1) * kFL + ci] - s_f[c][cj * kFL + ci];
            const double Dy = flux_quotient<FAST>(d, A.dx[1], A.rdx[1]);
            Lc[c] = -(Dx[c] + Dy);
        }
        if (A.has_grav) {
            // gravity source (Sec. 4.3, TEST 6) of the stage's input state
            const double rho = s_u[0][li];
            double e = 0.0;
#pragma unroll
            for (int d = 0; d < 2; ++d) {
                const double md = s_u[1 + d][li];
                Lc[1 + d] = Lc[1 + d] + (-(A.grav[d] * rho));
                e = d == 0 ? A.grav[0] * md : e + A.grav[d] * md;
            }
            Lc[3] = Lc[3] + (-e);
        }
        if constexpr (MODE == MODE_LAST_RHS) {
#pragma unroll
            for (int c = 0; c < M; ++c) A.out[c * ncell + idx] = Lc[c];
        } else {
            const double dt = st->dt;
            double un[M];
#pragma unroll
            for (int c = 0; c < M; ++c)
                un[c] = rk3_stage<FAST>(A.stage, s_u[c][li], Lc[c], dt, u0v[c]);
#pragma unroll
            for (int c = 0; c < M; ++c) A.out[c * ncell + idx] = un[c];
            double lam[6];
            err2 |= euler_speeds<2, FAST>(un, A.gamma, lam);
#pragma unroll
            for (int k = 0; k < NV; ++k) spd[k] = lam[k];
        }
    }
    if constexpr (MODE == MODE_LAST_STAGE) {
        if (err2) atomicOr(&st->err, err2);
        constexpr int NS = SpeedLayout<SYS_EULER, 2>::NS;
        int src[NS], sidx[NS];
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            src[j] = SpeedLayout<SYS_EULER, 2>::value_of_slot(j);
            sidx[j] = SpeedLayout<SYS_EULER, 2>::slot_index(j);
        }
        block_slot_max<NV, NS, kFThreads, true>(spd, st->alpha[A.slot_wr], src, sidx);
        if (blockIdx.x == 0 && t < kSlotLen)
            __hip_atomic_store(&st->alpha[A.slot_zero][t], 0ull, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
}

hipError_t launch_stage2d(int mode, int prec, const Stage2dArgs &A0, hipStream_t s)
{
    Stage2dArgs A = A0;
    A.ntx = (A.n[0] + kFX - 1) / kFX;
    A.tiles = A.ntx * ((A.n[1] + kFY - 1) / kFY);
    A.tiles_per_xcd = (A.tiles + kXcds - 1) / kXcds;
    const int64_t blocks = A.tiles_per_xcd * kXcds;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 g((unsigned)blocks), bl(kFThreads);
    const bool rhs = mode == MODE_LAST_RHS;
    if (prec == WT_FP32_RECON) {
        if (rhs) hipLaunchKernelGGL((stage2d_kernel<MODE_LAST_RHS, 1>), g, bl, 0, s, A);
        else hipLaunchKernelGGL((stage2d_kernel<MODE_LAST_STAGE, 1>), g, bl, 0, s, A);
    } else if (prec == WT_FP64_FAST) {
        if (rhs) hipLaunchKernelGGL((stage2d_kernel<MODE_LAST_RHS, 2>), g, bl, 0, s, A);
        else hipLaunchKernelGGL((stage2d_kernel<MODE_LAST_STAGE, 2>), g, bl, 0, s, A);
    } else {
        if (rhs) hipLaunchKernelGGL((stage2d_kernel<MODE_LAST_RHS, 0>), g, bl, 0, s, A);
        else hipLaunchKernelGGL((stage2d_kernel<MODE_LAST_STAGE, 0>), g, bl, 0, s, A);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Launch helpers
// ---------------------------------------------------------------------------
// Tile shapes (TX columns x TN points along the sweep, TX (TN + 1) = 256
// interfaces).  x-sweeps: 1 x 255 (a contiguous row segment).  y/z-sweeps of
// the Euler system in 2D/3D: one of kTileVariants shapes, chosen per grid by
// wenotheta_tune (default 0); every shape computes the same interface fluxes
// with the same operations, so the results do not depend on the choice.
//   0: 8 x 31   1: 16 x 15   2: 4 x 63   3: 32 x 7
template <int V>
struct TileYZ;
template <>
struct TileYZ<0> { static constexpr int TX = 8, TN = 31; };
template <>
struct TileYZ<1> { static constexpr int TX = 16, TN = 15; };
template <>
struct TileYZ<2> { static constexpr int TX = 4, TN = 63; };
template <>
struct TileYZ<3> { static constexpr int TX = 32, TN = 7; };

// x-sweeps of the Euler system in 2D/3D: 1 x 255 (one row segment; default) or
// 8 rows x 31 points, for rows whose length leaves a nearly empty last segment of
// 255 (a 512-point row: 255 + 255 + 2).  In 2D, variant 2 replaces the two sweeps
// of a stage by the fused stage kernel (stage2d_kernel).
//   0: 1 x 255   1: 8 x 31   2: fused 2D stage (2D only)
constexpr int kXTileVariants = 3;
constexpr int kXFused = 2;

template <int SYS, int NDIM, int DIR>
constexpr bool has_tile_variants()
{
    return SYS == SYS_EULER && NDIM > 1;
}

template <int SYS, int NDIM, int DIR, int MODE, int PREC, int TX, int TN>
hipError_t launch_tile(const SweepArgs &A, hipStream_t s)
{
    const int64_t nd = A.n[DIR];
    const int64_t nseg = (nd + TN - 1) / TN;
    int64_t blocks;
    if (DIR == 0) blocks = nseg * ((A.n[1] * A.n[2] + TX - 1) / TX);
    else if (DIR == 1) blocks = ((A.n[0] + TX - 1) / TX) * nseg * A.n[2];
    else blocks = ((A.n[0] + TX - 1) / TX) * nseg * A.n[1];
    SweepArgs B = A;
    if (DIR != 0) {
        B.tiles = blocks;
        B.tiles_per_xcd = (blocks + kXcds - 1) / kXcds;
        blocks = B.tiles_per_xcd * kXcds;
    }
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((sweep_kernel<SYS, NDIM, DIR, TX, TN, MODE, PREC>), dim3((unsigned)blocks),
                       dim3(kThreads), 0, s, B);
    return hipGetLastError();
}

template <int SYS, int NDIM, int DIR, int MODE, int PREC>
hipError_t launch_sweep(const SweepArgs &A, int tile, hipStream_t s)
{
    if constexpr (!has_tile_variants<SYS, NDIM, DIR>()) {
        (void)tile;
        constexpr int TX = DIR == 0 ? 1 : 8;
        constexpr int TN = DIR != 0 ? 31 : (split_fields<SYS, NDIM, PREC>() ? kThreads / Ncomp<SYS, NDIM>::value - 1 : 255);
        return launch_tile<SYS, NDIM, DIR, MODE, PREC, TX, TN>(A, s);
    } else if constexpr (DIR == 0) {
        if (tile == 1) return launch_tile<SYS, NDIM, DIR, MODE, PREC, TileYZ<0>::TX, TileYZ<0>::TN>(A, s);
        return launch_tile<SYS, NDIM, DIR, MODE, PREC, 1, 255>(A, s);   // 0 (and the fused 2)
    } else {
        switch (tile) {
            case 1: return launch_tile<SYS, NDIM, DIR, MODE, PREC, TileYZ<1>::TX, TileYZ<1>::TN>(A, s);
            case 2: return launch_tile<SYS, NDIM, DIR, MODE, PREC, TileYZ<2>::TX, TileYZ<2>::TN>(A, s);
            case 3: return launch_tile<SYS, NDIM, DIR, MODE, PREC, TileYZ<3>::TX, TileYZ<3>::TN>(A, s);
            default: return launch_tile<SYS, NDIM, DIR, MODE, PREC, TileYZ<0>::TX, TileYZ<0>::TN>(A, s);
        }
    }
}

template <int SYS, int NDIM, int DIR, int PREC>
hipError_t launch_sweep_mode(int mode, const SweepArgs &A, int tile, hipStream_t s)
{
    switch (mode) {
        case MODE_FIRST: return launch_sweep<SYS, NDIM, DIR, MODE_FIRST, PREC>(A, tile, s);
        case MODE_MID: return launch_sweep<SYS, NDIM, DIR, MODE_MID, PREC>(A, tile, s);
        case MODE_LAST_RHS: return launch_sweep<SYS, NDIM, DIR, MODE_LAST_RHS, PREC>(A, tile, s);
        default: return launch_sweep<SYS, NDIM, DIR, MODE_LAST_STAGE, PREC>(A, tile, s);
    }
}

template <int SYS, int NDIM, int PREC>
hipError_t launch_sweep_dir(int dir, int mode, const SweepArgs &A, int tile, hipStream_t s)
{
    if (dir == 0) return launch_sweep_mode<SYS, NDIM, 0, PREC>(mode, A, tile, s);
    if constexpr (NDIM > 1)
        if (dir == 1) return launch_sweep_mode<SYS, NDIM, 1, PREC>(mode, A, tile, s);
    if constexpr (NDIM > 2)
        if (dir == 2) return launch_sweep_mode<SYS, NDIM, 2, PREC>(mode, A, tile, s);
    return hipErrorInvalidValue;
}

template <int PREC>
hipError_t launch_sweep_prec(int sys, int ndim, int dir, int mode, const SweepArgs &A, int tile,
                             hipStream_t s)
{
    if (sys == SYS_LINEAR) return launch_sweep_dir<SYS_LINEAR, 1, PREC>(dir, mode, A, tile, s);
    if (sys == SYS_BURGERS) return launch_sweep_dir<SYS_BURGERS, 1, PREC>(dir, mode, A, tile, s);
    if (ndim == 1) return launch_sweep_dir<SYS_EULER, 1, PREC>(dir, mode, A, tile, s);
    if (ndim == 2) return launch_sweep_dir<SYS_EULER, 2, PREC>(dir, mode, A, tile, s);
    return launch_sweep_dir<SYS_EULER, 3, PREC>(dir, mode, A, tile, s);
}

hipError_t launch_sweep_any(int sys, int ndim, int prec, int dir, int mode, const SweepArgs &A,
                            int tile, hipStream_t s)
{
    if (prec == WT_FP32_RECON) return launch_sweep_prec<1>(sys, ndim, dir, mode, A, tile, s);
    if (prec == WT_FP64_FAST) return launch_sweep_prec<2>(sys, ndim, dir, mode, A, tile, s);
    return launch_sweep_prec<0>(sys, ndim, dir, mode, A, tile, s);
}

hipError_t launch_alpha(int sys, int ndim, const double *u, int64_t ncell, double a, double gamma,
                        DevState *st, int slot, hipStream_t s)
{
    int64_t blocks = (ncell + kThreads - 1) / kThreads;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    const dim3 g((unsigned)blocks), bl(kThreads);
    if (sys == SYS_LINEAR)
        hipLaunchKernelGGL((alpha_kernel<SYS_LINEAR, 1>), g, bl, 0, s, u, ncell, a, gamma, st, slot);
    else if (sys == SYS_BURGERS)
        hipLaunchKernelGGL((alpha_kernel<SYS_BURGERS, 1>), g, bl, 0, s, u, ncell, a, gamma, st, slot);
    else if (ndim == 1)
        hipLaunchKernelGGL((alpha_kernel<SYS_EULER, 1>), g, bl, 0, s, u, ncell, a, gamma, st, slot);
    else if (ndim == 2)
        hipLaunchKernelGGL((alpha_kernel<SYS_EULER, 2>), g, bl, 0, s, u, ncell, a, gamma, st, slot);
    else
        hipLaunchKernelGGL((alpha_kernel<SYS_EULER, 3>), g, bl, 0, s, u, ncell, a, gamma, st, slot);
    return hipGetLastError();
}

}  // namespace wt

// ---------------------------------------------------------------------------
// Context and C ABI
// ---------------------------------------------------------------------------
#include "wt_ctx.hpp"

namespace {

using namespace wt;

struct Shape {
    int ndim;
    int m;
    int64_t n[3];
    int64_t ncell;
    double dx[3];
    double lo[3];
    int bc[3];
    int walls[3];         // reflective ends, or a side with a wall part
    bool sides;           // some dimension is WT_SIDES
};

// sides: the side table WT_SIDES dimensions follow (null: none is set).
wt_status validate_grid(const wt_side *sides, const wt_grid *G, const wt_params *P, Shape &S)
{
    if (!G || !P) return WT_ERR_ARG;
    if (G->ndim < 1 || G->ndim > 3) return WT_ERR_ARG;
    S.sides = false;
    if (P->system < WT_LINEAR || P->system > WT_EULER) return WT_ERR_ARG;
    if (P->precision != WT_FP64 && P->precision != WT_FP32_RECON && P->precision != WT_FP64_FAST)
        return WT_ERR_ARG;
    if (P->system != WT_EULER && G->ndim != 1) return WT_ERR_UNSUPPORTED;
    if (!(P->cfl > 0.0) || !(P->eps > 0.0) || !(P->alpha_R >= 0.0)) return WT_ERR_ARG;
    if (P->system == WT_EULER && !(P->gamma > 1.0)) return WT_ERR_ARG;
    if (P->system == WT_LINEAR && !std::isfinite(P->a)) return WT_ERR_ARG;
    for (int d = 0; d < 3; ++d) {
        if (!std::isfinite(P->gravity[d])) return WT_ERR_ARG;
        if (P->gravity[d] != 0.0 && (P->system != WT_EULER || d >= G->ndim)) return WT_ERR_ARG;
    }
    S.ndim = G->ndim;
    S.m = P->system == WT_EULER ? G->ndim + 2 : 1;
    S.ncell = 1;
    for (int k = 0; k < 3; ++k) {
        if (k < G->ndim) {
            if (G->n[k] < 6 || G->n[k] > (int64_t(1) << 31)) return WT_ERR_ARG;
            if (!(G->hi[k] > G->lo[k])) return WT_ERR_ARG;
            if (G->bc[k] != WT_PERIODIC && G->bc[k] != WT_TRANSMISSIVE && G->bc[k] != WT_REFLECTIVE &&
                G->bc[k] != WT_SIDES)
                return WT_ERR_ARG;
            if ((G->bc[k] == WT_REFLECTIVE || G->bc[k] == WT_SIDES) && P->system != WT_EULER)
                return WT_ERR_UNSUPPORTED;
            if (G->bc[k] == WT_SIDES && !sides) return WT_ERR_ARG;
            S.n[k] = G->n[k];
            S.dx[k] = (G->hi[k] - G->lo[k]) / (double)G->n[k];
            S.lo[k] = G->lo[k];
            S.bc[k] = G->bc[k];
            S.walls[k] = G->bc[k] == WT_REFLECTIVE;
            if (G->bc[k] == WT_SIDES) {
                S.sides = true;
                for (int e = 0; e < 2; ++e)
                    for (int q = 0; q < 2; ++q)
                        S.walls[k] |= sides[2 * k + e].kind[q] == WT_SIDE_REFLECTIVE;
            }
        } else {
            if (G->n[k] != 1) return WT_ERR_ARG;
            S.n[k] = 1;
            S.dx[k] = 1.0;
            S.lo[k] = 0.0;
            S.bc[k] = WT_PERIODIC;
            S.walls[k] = 0;
        }
        S.ncell *= S.n[k];
    }
    if (S.ncell * S.m > (int64_t(1) << 40)) return WT_ERR_ARG;
    return WT_OK;
}

wt_status validate(const wt_ctx *c, const wt_grid *G, const wt_params *P, Shape &S)
{
    return validate_grid(c->has_sides ? c->sides : nullptr, G, P, S);
}

wt_status ensure_workspace(wt_ctx *c, const Shape &S)
{
    const size_t need = (size_t)S.ncell * (size_t)S.m;
    if (need <= c->cap) return WT_OK;
    if (hipSetDevice(c->device) != hipSuccess) return WT_ERR_DEVICE;
    (void)hipFree(c->U1);
    (void)hipFree(c->U2);
    (void)hipFree(c->D);
    c->U1 = c->U2 = c->D = nullptr;
    c->cap = 0;
    if (hipMalloc(&c->U1, need * sizeof(double)) != hipSuccess ||
        hipMalloc(&c->U2, need * sizeof(double)) != hipSuccess ||
        hipMalloc(&c->D, need * sizeof(double)) != hipSuccess) {
        (void)hipFree(c->U1);
        (void)hipFree(c->U2);
        (void)hipFree(c->D);
        c->U1 = c->U2 = c->D = nullptr;
        (void)hipGetLastError();
        return WT_ERR_NOMEM;
    }
    c->cap = need;
    return WT_OK;
}

uint64_t bits(double d)
{
    uint64_t b;
    std::memcpy(&b, &d, sizeof b);
    return b;
}

uint64_t plan_key(const Shape &S, const wt_params *P)
{
    uint64_t h = 1469598103934665603ull;
    for (uint64_t v : {(uint64_t)P->system, (uint64_t)S.ndim, (uint64_t)S.n[0], (uint64_t)S.n[1],
                       (uint64_t)S.n[2], (uint64_t)P->precision})
        h = (h ^ v) * 1099511628211ull;
    return h;
}

// Tile variant of direction dir for this grid (0 unless tuned or set).
int plan_tile(const wt_ctx *c, const Shape &S, const wt_params *P, int dir)
{
    const uint64_t key = plan_key(S, P);
    for (int i = 0; i < c->nplans; ++i)
        if (c->plans[i].key == key) return c->plans[i].tile[dir];
    return 0;
}

bool fused_stage(const wt_ctx *c, const Shape &S, const wt_params *P)
{
    return P->system == WT_EULER && S.ndim == 2 && !S.sides && plan_tile(c, S, P, 0) == kXFused;
}

void set_plan(wt_ctx *c, const Shape &S, const wt_params *P, const int *tile)
{
    const uint64_t key = plan_key(S, P);
    int i = 0;
    while (i < c->nplans && c->plans[i].key != key) ++i;
    if (i == c->nplans) i = c->nplans < kTilePlans ? c->nplans++ : kTilePlans - 1;
    for (; i > 0; --i) c->plans[i] = c->plans[i - 1];          // most recent first
    c->plans[0].key = key;
    for (int d = 0; d < 3; ++d) c->plans[0].tile[d] = (int8_t)tile[d];
}

// Launch one kernel, bracketed by profiling events of the given kind when enabled.
template <class Launch>
hipError_t timed_launch(wt_ctx *c, int kind, hipStream_t s, Launch launch)
{
    const bool rec = c->prof && c->nev < kProfPairs;
    if (c->prof && !rec) c->prof_dropped++;
    if (rec && hipEventRecord(c->ev[2 * c->nev], s) != hipSuccess) return hipErrorUnknown;
    const hipError_t e = launch();
    if (e != hipSuccess) return e;
    if (rec) {
        if (hipEventRecord(c->ev[2 * c->nev + 1], s) != hipSuccess) return hipErrorUnknown;
        c->ev_kind[c->nev] = kind;
        c->nev++;
    }
    return hipSuccess;
}

// Launch one sweep, bracketed by profiling events when enabled.
hipError_t timed_sweep(wt_ctx *c, int sys, int ndim, int prec, int dir, int mode,
                       const SweepArgs &A, int tile, hipStream_t s)
{
    const int kind = (mode == MODE_LAST_RHS || mode == MODE_LAST_STAGE ? 3 : 0) + dir;
    return timed_launch(c, kind, s, [&] { return launch_sweep_any(sys, ndim, prec, dir, mode, A, tile, s); });
}

// Whether the stages of this grid run as the fused 2D stage kernel.
bool fused_stage(const wt_ctx *c, const Shape &S, const wt_params *P);

// The fused kernel's arguments from a sweep's (speed slots, stage, buffers).
Stage2dArgs stage2d_args(const wt_ctx *c, const Shape &S, const wt_params *P, const SweepArgs &B)
{
    Stage2dArgs A{};
    A.uin = B.uin;
    A.u0 = B.u0;
    A.out = B.out;
    A.st = B.st;
    A.n[0] = S.n[0];
    A.n[1] = S.n[1];
    A.ncell = S.ncell;
    for (int d = 0; d < 2; ++d) {
        A.dx[d] = S.dx[d];
        A.rdx[d] = 1.0 / S.dx[d];
        A.bc[d] = S.bc[d];
        A.walls[d] = S.walls[d];
        A.grav[d] = P->gravity[d];
    }
    A.gamma = P->gamma;
    A.W = B.W;
    A.slot_rd = B.slot_rd;
    A.slot_wr = B.slot_wr;
    A.slot_zero = B.slot_zero;
    A.stage = B.stage;
    A.check_done = B.check_done;
    A.has_grav = B.has_grav;
    (void)c;
    return A;
}

// Fold the recorded (completed) event pairs into the per-kind totals.
void drain_profile(wt_ctx *c)
{
    for (int k = 0; k < c->nev; ++k) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]) == hipSuccess) {
            c->prof_ms[c->ev_kind[k]] += ms;
            c->prof_n[c->ev_kind[k]] += 1;
        }
    }
    c->nev = 0;
}

SweepArgs base_args(DevState *st, double *D, const Shape &S, const wt_params *P)
{
    SweepArgs A{};
    A.st = st;
    for (int k = 0; k < 3; ++k) A.n[k] = S.n[k];
    A.ncell = S.ncell;
    A.a = P->a;
    A.gamma = P->gamma;
    A.W = WenoConst{P->eps, P->alpha_R, 1.0 / P->eps};
    A.D = D;
    for (int d = 0; d < 3; ++d) {
        A.grav[d] = P->gravity[d];
        A.has_grav |= P->gravity[d] != 0.0;
    }
    return A;
}

SweepArgs base_args(wt_ctx *c, const Shape &S, const wt_params *P)
{
    return base_args(c->st, c->D, S, P);
}

// The arguments of a sweep along direction d.
void dir_args(SweepArgs &A, const wt_side *sides, const Shape &S, int d)
{
    A.dx = S.dx[d];
    A.rdx = 1.0 / S.dx[d];
    A.bc = S.bc[d];
    A.walls = S.walls[d];
    if (S.bc[d] == WT_SIDES) {
        const int a = (d + 1) % S.ndim;
        A.side[0] = sides[2 * d];
        A.side[1] = sides[2 * d + 1];
        A.tlo = S.lo[a];
        A.tdx = S.dx[a];
    }
}

void dir_args(SweepArgs &A, const wt_ctx *c, const Shape &S, int d)
{
    dir_args(A, c->sides, S, d);
}

// Queue the speeds of u into slot g % 3 and zero slot (g + 1) % 3.
wt_status queue_alpha_init(wt_ctx *c, const Shape &S, const wt_params *P, const double *u,
                           hipStream_t s)
{
    const int rd = (int)(c->g % kSlots), nx = (int)((c->g + 1) % kSlots);
    SlotValues zero{};
    hipLaunchKernelGGL(set_slots_kernel, dim3(1), dim3(64), 0, s, c->st, rd, zero, nx);
    if (hipGetLastError() != hipSuccess) return WT_ERR_DEVICE;
    if (launch_alpha(P->system, S.ndim, u, S.ncell, P->a, P->gamma, c->st, rd, s) != hipSuccess)
        return WT_ERR_DEVICE;
    return WT_OK;
}

// One Runge-Kutta stage: uin -> out, reading speeds of uin from slot g % 3 and
// writing those of out into slot (g + 1) % 3.
wt_status queue_stage(wt_ctx *c, const Shape &S, const wt_params *P, const double *uin,
                      const double *u0, double *out, int stage, hipStream_t s)
{
    SweepArgs A = base_args(c, S, P);
    A.uin = uin;
    A.u0 = u0;
    A.out = out;
    A.stage = stage;
    A.check_done = 1;
    A.slot_rd = (int)(c->g % kSlots);
    A.slot_wr = (int)((c->g + 1) % kSlots);
    A.slot_zero = (int)((c->g + 2) % kSlots);
    if (fused_stage(c, S, P)) {
        const Stage2dArgs F = stage2d_args(c, S, P, A);
        if (timed_launch(c, kProfFused, s, [&] { return launch_stage2d(MODE_LAST_STAGE, P->precision, F, s); }) !=
            hipSuccess)
            return WT_ERR_DEVICE;
        c->g += 1;
        return WT_OK;
    }
    for (int d = 0; d < S.ndim; ++d) {
        const int mode = d == S.ndim - 1 ? MODE_LAST_STAGE : (d == 0 ? MODE_FIRST : MODE_MID);
        dir_args(A, c, S, d);
        if (timed_sweep(c, P->system, S.ndim, P->precision, d, mode, A, plan_tile(c, S, P, d), s) !=
            hipSuccess)
            return WT_ERR_DEVICE;
    }
    c->g += 1;
    return WT_OK;
}

wt_status queue_step(wt_ctx *c, const Shape &S, const wt_params *P, double *u, double dt_fixed,
                     int clip, hipStream_t s)
{
    StepArgs B{};
    B.st = c->st;
    B.slot = (int)(c->g % kSlots);
    B.ndim = S.ndim;
    B.euler = P->system == WT_EULER;
    for (int k = 0; k < 3; ++k) B.dx[k] = S.dx[k];
    B.cfl = P->cfl;
    B.dt_fixed = dt_fixed;
    B.clip = clip;
    hipLaunchKernelGGL(step_begin_kernel, dim3(1), dim3(64), 0, s, B);
    if (hipGetLastError() != hipSuccess) return WT_ERR_DEVICE;
    wt_status r;
    if ((r = queue_stage(c, S, P, u, u, c->U1, 1, s))) return r;
    if ((r = queue_stage(c, S, P, c->U1, u, c->U2, 2, s))) return r;
    if ((r = queue_stage(c, S, P, c->U2, u, u, 3, s))) return r;
    return WT_OK;
}

// The solver graph: kGraphSteps steps of the current grid captured once per
// argument set and replayed.  A step advances the stage counter by 3, so the
// speed slots every replay uses are those of the capture.
wt_status ensure_step_graph(wt_ctx *c, const Shape &S, const wt_params *P, double *u)
{
    uint64_t key = plan_key(S, P);
    for (uint64_t v : {(uint64_t)(uintptr_t)u, (uint64_t)(uintptr_t)c->U1, (uint64_t)(uintptr_t)c->U2,
                       (uint64_t)(uintptr_t)c->D, (uint64_t)(uintptr_t)c->st, (uint64_t)(c->g % kSlots),
                       (uint64_t)plan_tile(c, S, P, 0), (uint64_t)plan_tile(c, S, P, 1), (uint64_t)plan_tile(c, S, P, 2), bits(P->a),
                       bits(P->gamma), bits(P->cfl), bits(P->eps), bits(P->alpha_R),
                       bits(P->gravity[0]), bits(P->gravity[1]), bits(P->gravity[2]), bits(S.dx[0]),
                       bits(S.dx[1]), bits(S.dx[2]), (uint64_t)S.bc[0], (uint64_t)S.bc[1], (uint64_t)S.bc[2]})
        key = (key ^ v) * 1099511628211ull;
    if (S.sides) {
        // the side table and the split axes' origins are captured in the sweeps' arguments
        const unsigned char *b = reinterpret_cast<const unsigned char *>(c->sides);
        for (size_t i = 0; i < sizeof c->sides; ++i) key = (key ^ b[i]) * 1099511628211ull;
        for (int k = 0; k < 3; ++k) key = (key ^ bits(S.lo[k])) * 1099511628211ull;
    }
    if (c->s_graph && c->s_key == key) return WT_OK;
    if (c->s_graph) (void)hipGraphExecDestroy(c->s_graph);
    c->s_graph = nullptr;
    if (!c->s_capture && hipStreamCreateWithFlags(&c->s_capture, hipStreamNonBlocking) != hipSuccess)
        return WT_ERR_DEVICE;
    if (hipStreamBeginCapture(c->s_capture, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return WT_ERR_DEVICE;
    const int64_t g0 = c->g;
    wt_status r = WT_OK;
    for (int i = 0; i < kGraphSteps && r == WT_OK; ++i) r = queue_step(c, S, P, u, 0.0, 1, c->s_capture);
    c->g = g0;
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(c->s_capture, &g);
    if (r != WT_OK || ec != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return r != WT_OK ? r : WT_ERR_DEVICE;
    }
    const hipError_t ei = hipGraphInstantiate(&c->s_graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
        c->s_graph = nullptr;
        return WT_ERR_DEVICE;
    }
    c->s_key = key;
    return WT_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Fixed scratch of wenotheta_rhs_noalloc
// ---------------------------------------------------------------------------
// One device array per GPU holds the device state (speed slot, error word) at
// offset 0 and the divergence accumulator of multi-dimensional grids after it.
// Host code never names the array in a kernel argument or a copy: it uses the
// address hipGetSymbolAddress returns on each device (the name is a host-side
// stand-in there).
namespace wt {
constexpr size_t kNoAllocBytes = size_t(64) << 20;
constexpr size_t kNoAllocStateBytes = 4096;   // DevState, padded so D stays aligned
static_assert(sizeof(DevState) <= kNoAllocStateBytes, "device state fits its part");
static_assert(sizeof(DevState) % sizeof(unsigned long long) == 0, "cleared word by word");
constexpr int64_t kNoAllocDoubles = (int64_t)((kNoAllocBytes - kNoAllocStateBytes) / sizeof(double));
constexpr int kNoAllocMaxDevices = 64;
}  // namespace wt

static __device__ __align__(256) unsigned char scratch[wt::kNoAllocBytes];

namespace {

using namespace wt;

std::mutex g_scratch_mu;
void *g_scratch_ptr[kNoAllocMaxDevices] = {};

// Device address of `scratch` on device dev (current), looked up on the first
// call for that device and kept.
wt_status noalloc_scratch(int dev, unsigned char **out)
{
    if (dev < 0 || dev >= kNoAllocMaxDevices) return WT_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return WT_ERR_DEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<unsigned char *>(g_scratch_ptr[dev]);
    return WT_OK;
}

// Zero the device state word by word (a kernel, not a memset node, so the
// call may be captured into a graph).
__global__ void clear_state_kernel(DevState *st)
{
    unsigned long long *w = reinterpret_cast<unsigned long long *>(st);
    for (int k = threadIdx.x; k < (int)(sizeof(DevState) / sizeof(unsigned long long)); k += blockDim.x)
        w[k] = 0ull;
}

// The status the device recorded, as a wt_status.
__global__ void status_kernel(const DevState *st, int32_t *out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const int e = st->err;
        *out = (e & kErrNonfinite) ? WT_ERR_NONFINITE : ((e & kErrNonphysical) ? WT_ERR_NONPHYSICAL : WT_OK);
    }
}

}  // namespace

namespace wt {

// Read and clear the device error word (synchronises the stream).
wt_status collect(wt_ctx *c, hipStream_t s, DevState *host)
{
    if (hipMemcpyAsync(host, c->st, sizeof(DevState), hipMemcpyDeviceToHost, s) != hipSuccess)
        return WT_ERR_DEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return WT_ERR_DEVICE;
    drain_profile(c);
    int e = host->err;
    if (e) {
        const int zero = 0;
        if (hipMemcpyAsync(&c->st->err, &zero, sizeof(int), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return WT_ERR_DEVICE;
    }
    if (e & kErrNonfinite) return WT_ERR_NONFINITE;
    if (e & kErrNonphysical) return WT_ERR_NONPHYSICAL;
    return WT_OK;
}

}  // namespace wt

extern "C" {

const char *wenotheta_status_string(int32_t s)
{
    switch (s) {
        case WT_OK: return "ok";
        case WT_ERR_ARG: return "invalid argument";
        case WT_ERR_UNSUPPORTED: return "unsupported configuration";
        case WT_ERR_NONPHYSICAL: return "non-physical state (rho <= 0 or p <= 0)";
        case WT_ERR_NONFINITE: return "non-finite value";
        case WT_ERR_DEVICE: return "HIP device error";
        case WT_ERR_NOMEM: return "out of device memory";
        case WT_ERR_SCRATCH: return "input larger than the fixed scratch buffer of wenotheta_rhs_noalloc";
        default: return "unknown status";
    }
}

wt_status wenotheta_ctx_create(wt_ctx **out, int32_t device)
{
    if (!out) return WT_ERR_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return WT_ERR_ARG;
    if (hipSetDevice(device) != hipSuccess) return WT_ERR_DEVICE;
    wt_ctx *c = new (std::nothrow) wt_ctx();
    if (!c) return WT_ERR_NOMEM;
    c->device = device;
    if (hipMalloc(&c->st, sizeof(DevState)) != hipSuccess) {
        delete c;
        return WT_ERR_NOMEM;
    }
    if (hipMemset(c->st, 0, sizeof(DevState)) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        (void)hipFree(c->st);
        delete c;
        return WT_ERR_DEVICE;
    }
    *out = c;
    return WT_OK;
}

wt_status wenotheta_ctx_destroy(wt_ctx *c)
{
    if (!c) return WT_ERR_ARG;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(c->U1);
    (void)hipFree(c->U2);
    (void)hipFree(c->D);
    (void)hipFree(c->st);
    for (int k = 0; k < 2 * kProfPairs; ++k)
        if (c->ev[k]) (void)hipEventDestroy(c->ev[k]);
    if (c->s_graph) (void)hipGraphExecDestroy(c->s_graph);
    if (c->s_capture) (void)hipStreamDestroy(c->s_capture);
    wt::release_batched(c);
    delete c;
    return WT_OK;
}

wt_status wenotheta_profile(wt_ctx *c, int32_t enable)
{
    if (!c) return WT_ERR_ARG;
    if (hipSetDevice(c->device) != hipSuccess) return WT_ERR_DEVICE;
    if (enable && !c->ev[0]) {
        for (int k = 0; k < 2 * kProfPairs; ++k)
            if (hipEventCreate(&c->ev[k]) != hipSuccess) return WT_ERR_DEVICE;
    }
    c->prof = enable != 0;
    c->nev = 0;
    for (int k = 0; k < kProfKinds; ++k) {
        c->prof_ms[k] = 0.0;
        c->prof_n[k] = 0;
    }
    c->prof_dropped = 0;
    return WT_OK;
}

wt_status wenotheta_profile_read(wt_ctx *c, double *ms, int64_t *count, int32_t nkinds)
{
    if (!c || !ms || !count || nkinds < 6) return WT_ERR_ARG;
    for (int k = 0; k < kProfKinds && k < nkinds; ++k) {
        ms[k] = c->prof_ms[k];
        count[k] = c->prof_n[k];
    }
    return c->prof_dropped ? WT_ERR_ARG : WT_OK;
}

wt_status wenotheta_rhs(wt_ctx *c, const wt_grid *G, const wt_params *P, const double *u,
                        const double *f, const double *alpha_host, double *L, void *stream)
{
    if (!c || !u || !L) return WT_ERR_ARG;
    Shape S;
    wt_status r = validate(c, G, P, S);
    if (r) return r;
    if (f && (P->system == WT_EULER || !alpha_host)) return WT_ERR_ARG;
    if (alpha_host)
        for (int k = 0; k < S.ndim * S.m; ++k)
            if (!(alpha_host[k] >= 0.0) || !std::isfinite(alpha_host[k])) return WT_ERR_ARG;
    if (hipSetDevice(c->device) != hipSuccess) return WT_ERR_DEVICE;
    if ((r = ensure_workspace(c, S))) return r;
    hipStream_t s = (hipStream_t)stream;
    if (alpha_host) {
        SlotValues v{};
        for (int d = 0; d < S.ndim; ++d)
            for (int k = 0; k < S.m; ++k) v.v[d * 5 + k] = alpha_host[d * S.m + k];
        hipLaunchKernelGGL(set_slots_kernel, dim3(1), dim3(64), 0, s, c->st, (int)(c->g % kSlots), v, -1);
        if (hipGetLastError() != hipSuccess) return WT_ERR_DEVICE;
    } else if ((r = queue_alpha_init(c, S, P, u, s))) {
        return r;
    }
    SweepArgs A = base_args(c, S, P);
    A.uin = u;
    A.out = L;
    A.fgiven = f;
    A.check_done = 0;
    A.slot_rd = (int)(c->g % kSlots);
    if (fused_stage(c, S, P)) {
        const Stage2dArgs F = stage2d_args(c, S, P, A);
        if (timed_launch(c, kProfFused, s, [&] { return launch_stage2d(MODE_LAST_RHS, P->precision, F, s); }) !=
            hipSuccess)
            return WT_ERR_DEVICE;
        return WT_OK;
    }
    for (int d = 0; d < S.ndim; ++d) {
        const int mode = d == S.ndim - 1 ? MODE_LAST_RHS : (d == 0 ? MODE_FIRST : MODE_MID);
        dir_args(A, c, S, d);
        if (timed_sweep(c, P->system, S.ndim, P->precision, d, mode, A, plan_tile(c, S, P, d), s) !=
            hipSuccess)
            return WT_ERR_DEVICE;
    }
    return WT_OK;
}

wt_status wenotheta_step(wt_ctx *c, const wt_grid *G, const wt_params *P, double *u, double dt,
                         double *dt_used, void *stream)
{
    if (!c || !u) return WT_ERR_ARG;
    Shape S;
    wt_status r = validate(c, G, P, S);
    if (r) return r;
    if (!std::isfinite(dt)) return WT_ERR_ARG;
    if (hipSetDevice(c->device) != hipSuccess) return WT_ERR_DEVICE;
    if ((r = ensure_workspace(c, S))) return r;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(solve_init_kernel, dim3(1), dim3(64), 0, s, c->st, 0.0, 0.0, -1ll, 0);
    if (hipGetLastError() != hipSuccess) return WT_ERR_DEVICE;
    if ((r = queue_alpha_init(c, S, P, u, s))) return r;
    if ((r = queue_step(c, S, P, u, dt > 0.0 ? dt : 0.0, 0, s))) return r;
    if (dt_used) {
        hipLaunchKernelGGL(copy_dt_kernel, dim3(1), dim3(64), 0, s, c->st, dt_used);
        if (hipGetLastError() != hipSuccess) return WT_ERR_DEVICE;
    }
    return WT_OK;
}

wt_status wenotheta_solve(wt_ctx *c, const wt_grid *G, const wt_params *P, double *u, double t0,
                          double t_end, int64_t max_steps, double *t_out, int64_t *steps_out,
                          void *stream)
{
    if (!c || !u) return WT_ERR_ARG;
    Shape S;
    wt_status r = validate(c, G, P, S);
    if (r) return r;
    if (std::isnan(t0) || std::isnan(t_end) || !std::isfinite(t0)) return WT_ERR_ARG;
    if (!std::isfinite(t_end) && max_steps < 0) return WT_ERR_ARG;
    if (hipSetDevice(c->device) != hipSuccess) return WT_ERR_DEVICE;
    if ((r = ensure_workspace(c, S))) return r;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(solve_init_kernel, dim3(1), dim3(64), 0, s, c->st, t0, t_end,
                       (long long)max_steps, 1);
    if (hipGetLastError() != hipSuccess) return WT_ERR_DEVICE;
    if ((r = queue_alpha_init(c, S, P, u, s))) return r;
    // Steps are queued in chunks (1, 2, 4, .. 64 steps) with one synchronisation
    // per chunk; steps past the end are no-ops on the device.  Without the
    // profiler the steps are replayed from a captured graph of kGraphSteps.
    const bool graph = !c->prof;
    if (graph && (r = ensure_step_graph(c, S, P, u))) return r;
    DevState host{};
    int64_t launched = 0;
    int64_t chunk = graph ? kGraphSteps : 1;
    for (;;) {
        int64_t k = chunk;
        if (max_steps >= 0 && launched + k > max_steps) k = max_steps - launched;
        if (graph) {
            for (int64_t i = 0; i < k; i += kGraphSteps) {
                if (hipGraphLaunch(c->s_graph, s) != hipSuccess) return WT_ERR_DEVICE;
                c->g += 3 * kGraphSteps;
            }
        } else {
            for (int64_t i = 0; i < k; ++i)
                if ((r = queue_step(c, S, P, u, 0.0, 1, s))) return r;
        }
        launched += k;
        if ((r = collect(c, s, &host))) return r;
        if (host.done || (max_steps >= 0 && launched >= max_steps)) break;
        if (chunk < 64) chunk *= 2;
    }
    if (t_out) *t_out = host.t;
    if (steps_out) *steps_out = host.steps;
    return WT_OK;
}

wt_status wenotheta_set_sides(wt_ctx *c, const wt_side *sides, double t, void *stream)
{
    if (!c || !std::isfinite(t)) return WT_ERR_ARG;
    if (sides) {
        for (int i = 0; i < 6; ++i) {
            const wt_side &e = sides[i];
            if (std::isnan(e.split0) || !std::isfinite(e.split_speed)) return WT_ERR_ARG;
            for (int q = 0; q < 2; ++q) {
                if (e.kind[q] != WT_SIDE_TRANSMISSIVE && e.kind[q] != WT_SIDE_REFLECTIVE &&
                    e.kind[q] != WT_SIDE_STATE)
                    return WT_ERR_ARG;
                if (e.kind[q] == WT_SIDE_STATE)
                    for (int k = 0; k < 5; ++k)
                        if (!std::isfinite(e.state[q][k])) return WT_ERR_ARG;
            }
        }
    }
    if (hipSetDevice(c->device) != hipSuccess) return WT_ERR_DEVICE;
    hipLaunchKernelGGL(set_time_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, c->st, t);
    if (hipGetLastError() != hipSuccess) return WT_ERR_DEVICE;
    if (sides) {
        for (int i = 0; i < 6; ++i) c->sides[i] = sides[i];
        c->has_sides = true;
    } else {
        c->has_sides = false;
    }
    return WT_OK;
}

wt_status wenotheta_set_tiles(wt_ctx *c, const wt_grid *G, const wt_params *P, const int32_t *tile)
{
    if (!c || !tile) return WT_ERR_ARG;
    Shape S;
    wt_status r = validate(c, G, P, S);
    if (r) return r;
    int t[3] = {0, 0, 0};
    for (int d = 0; d < S.ndim; ++d) {
        if (tile[d] < 0 || tile[d] >= (d == 0 ? kXTileVariants : kTileVariants)) return WT_ERR_ARG;
        if (d == 0 && tile[d] == kXFused && !(P->system == WT_EULER && S.ndim == 2 && !S.sides))
            return WT_ERR_ARG;
        t[d] = tile[d];
    }
    set_plan(c, S, P, t);
    return WT_OK;
}

wt_status wenotheta_tune(wt_ctx *c, const wt_grid *G, const wt_params *P, const double *u,
                         int32_t *tile_out, void *stream)
{
    if (!c || !u) return WT_ERR_ARG;
    Shape S;
    wt_status r = validate(c, G, P, S);
    if (r) return r;
    if (hipSetDevice(c->device) != hipSuccess) return WT_ERR_DEVICE;
    if ((r = ensure_workspace(c, S))) return r;
    hipStream_t s = (hipStream_t)stream;
    int best[3] = {0, 0, 0};
    if (P->system == WT_EULER && S.ndim > 1) {
        // Each direction is timed in the role a step gives it (first, accumulating or
        // stage-finishing sweep), on u, with the stage written to the workspace U2:
        // set up a CFL dt from the speeds of u, then the divergence of the earlier
        // directions, as the stage would.
        hipLaunchKernelGGL(solve_init_kernel, dim3(1), dim3(64), 0, s, c->st, 0.0, 0.0, -1ll, 0);
        if (hipGetLastError() != hipSuccess) return WT_ERR_DEVICE;
        if ((r = queue_alpha_init(c, S, P, u, s))) return r;
        StepArgs B{};
        B.st = c->st;
        B.slot = (int)(c->g % kSlots);
        B.ndim = S.ndim;
        B.euler = 1;
        for (int k = 0; k < 3; ++k) B.dx[k] = S.dx[k];
        B.cfl = P->cfl;
        hipLaunchKernelGGL(step_begin_kernel, dim3(1), dim3(64), 0, s, B);
        if (hipGetLastError() != hipSuccess) return WT_ERR_DEVICE;
        SweepArgs A = base_args(c, S, P);
        A.uin = u;
        A.u0 = u;
        A.out = c->U2;
        A.stage = 1;
        A.check_done = 0;
        A.slot_rd = (int)(c->g % kSlots);
        A.slot_wr = (int)((c->g + 1) % kSlots);
        A.slot_zero = (int)((c->g + 2) % kSlots);
        auto args_for = [&](int d) {
            dir_args(A, c, S, d);
            return d == S.ndim - 1 ? MODE_LAST_STAGE : (d == 0 ? MODE_FIRST : MODE_MID);
        };
        hipEvent_t e0, e1;
        if (hipEventCreate(&e0) != hipSuccess) return WT_ERR_DEVICE;
        if (hipEventCreate(&e1) != hipSuccess) {
            (void)hipEventDestroy(e0);
            return WT_ERR_DEVICE;
        }
        for (int d = 0; d < S.ndim && r == WT_OK; ++d) {
            const int nvar = d == 0 ? kXFused : kTileVariants;      // the sweep shapes
            // the divergence of the directions before d, as the stage forms it
            // (an accumulating sweep timed for an earlier direction added to it
            // several times)
            for (int e = 0; e < d && r == WT_OK; ++e) {
                const int me = args_for(e);
                if (launch_sweep_any(P->system, S.ndim, P->precision, e, me, A, best[e], s) != hipSuccess)
                    r = WT_ERR_DEVICE;
            }
            const int mode = args_for(d);
            {
                // candidates interleaved over rounds; each keeps its fastest launch
                float ms_best[kTileVariants];
                for (int v = 0; v < kTileVariants; ++v) ms_best[v] = 1e30f;
                for (int round = 0; round < 4 && r == WT_OK; ++round)
                    for (int v = 0; v < nvar && r == WT_OK; ++v) {
                        float ms = 0.0f;
                        if (hipEventRecord(e0, s) != hipSuccess ||
                            launch_sweep_any(P->system, S.ndim, P->precision, d, mode, A, v, s) != hipSuccess ||
                            hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                            r = WT_ERR_DEVICE;
                            break;
                        }
                        if (round > 0 && ms < ms_best[v]) ms_best[v] = ms;   // round 0 warms up
                    }
                // another shape replaces the default only if clearly faster
                for (int v = 1; v < nvar; ++v)
                    if (ms_best[v] < 0.98f * ms_best[0] && ms_best[v] < ms_best[best[d]]) best[d] = v;
            }
        }
        // 2D: a whole stage by the fused kernel against the two chosen sweeps queued
        // back to back, rounds interleaved (it replaces the pair only if clearly faster)
        if (r == WT_OK && S.ndim == 2 && !S.sides) {
            SweepArgs Bx = A, By = A;
            dir_args(Bx, c, S, 0);
            dir_args(By, c, S, 1);
            const Stage2dArgs F = stage2d_args(c, S, P, By);
            float ms_pair = 1e30f, ms_f = 1e30f;
            for (int round = 0; round < 5 && r == WT_OK; ++round)
                for (int v = 0; v < 2 && r == WT_OK; ++v) {
                    float ms = 0.0f;
                    hipError_t e = hipEventRecord(e0, s);
                    if (e == hipSuccess && v == 0) {
                        e = launch_sweep_any(P->system, 2, P->precision, 0, MODE_FIRST, Bx, best[0], s);
                        if (e == hipSuccess)
                            e = launch_sweep_any(P->system, 2, P->precision, 1, MODE_LAST_STAGE, By, best[1], s);
                    } else if (e == hipSuccess) {
                        e = launch_stage2d(MODE_LAST_STAGE, P->precision, F, s);
                    }
                    if (e != hipSuccess || hipEventRecord(e1, s) != hipSuccess ||
                        hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                        r = WT_ERR_DEVICE;
                        break;
                    }
                    float &m = v == 0 ? ms_pair : ms_f;
                    if (round > 0 && ms < m) m = ms;          // round 0 warms up
                }
            if (ms_f < 0.98f * ms_pair) best[0] = kXFused;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (r) return r;
        hipLaunchKernelGGL(restore_time_kernel, dim3(1), dim3(64), 0, s, c->st);
        if (hipGetLastError() != hipSuccess) return WT_ERR_DEVICE;
    }
    set_plan(c, S, P, best);
    if (tile_out)
        for (int d = 0; d < S.ndim; ++d) tile_out[d] = best[d];
    DevState host{};
    return collect(c, s, &host);
}

wt_status wenotheta_sync(wt_ctx *c, void *stream)
{
    if (!c) return WT_ERR_ARG;
    if (hipSetDevice(c->device) != hipSuccess) return WT_ERR_DEVICE;
    DevState host{};
    return collect(c, (hipStream_t)stream, &host);
}

wt_status wenotheta_rhs_noalloc(const wt_grid *G, const wt_params *P, const double *u,
                                const double *f, const double *alpha_host, double *L,
                                int32_t *status_dev, void *stream)
{
    if (!u || !L || !G) return WT_ERR_ARG;
    for (int k = 0; k < G->ndim && k < 3; ++k)
        if (G->bc[k] == WT_SIDES) return WT_ERR_UNSUPPORTED;   // no side table without a context
    Shape S;
    wt_status r = validate_grid(nullptr, G, P, S);
    if (r) return r;
    if (f && (P->system == WT_EULER || !alpha_host)) return WT_ERR_ARG;
    if (alpha_host)
        for (int k = 0; k < S.ndim * S.m; ++k)
            if (!(alpha_host[k] >= 0.0) || !std::isfinite(alpha_host[k])) return WT_ERR_ARG;
    // the divergence accumulator of a multi-dimensional grid must fit the buffer
    if (S.ndim > 1 && S.ncell * S.m > kNoAllocDoubles) return WT_ERR_SCRATCH;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return WT_ERR_DEVICE;
    unsigned char *base = nullptr;
    if ((r = noalloc_scratch(dev, &base))) return r;
    DevState *st = reinterpret_cast<DevState *>(base);
    double *D = reinterpret_cast<double *>(base + kNoAllocStateBytes);
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(clear_state_kernel, dim3(1), dim3(64), 0, s, st);
    if (hipGetLastError() != hipSuccess) return WT_ERR_DEVICE;
    if (alpha_host) {
        SlotValues v{};
        for (int d = 0; d < S.ndim; ++d)
            for (int k = 0; k < S.m; ++k) v.v[d * 5 + k] = alpha_host[d * S.m + k];
        hipLaunchKernelGGL(set_slots_kernel, dim3(1), dim3(64), 0, s, st, 0, v, -1);
        if (hipGetLastError() != hipSuccess) return WT_ERR_DEVICE;
    } else if (launch_alpha(P->system, S.ndim, u, S.ncell, P->a, P->gamma, st, 0, s) != hipSuccess) {
        return WT_ERR_DEVICE;
    }
    SweepArgs A = base_args(st, D, S, P);
    A.uin = u;
    A.out = L;
    A.fgiven = f;
    A.check_done = 0;
    A.slot_rd = 0;
    for (int d = 0; d < S.ndim; ++d) {
        const int mode = d == S.ndim - 1 ? MODE_LAST_RHS : (d == 0 ? MODE_FIRST : MODE_MID);
        dir_args(A, static_cast<const wt_side *>(nullptr), S, d);
        if (launch_sweep_any(P->system, S.ndim, P->precision, d, mode, A, 0, s) != hipSuccess)
            return WT_ERR_DEVICE;
    }
    if (status_dev) {
        hipLaunchKernelGGL(status_kernel, dim3(1), dim3(64), 0, s, st, status_dev);
        if (hipGetLastError() != hipSuccess) return WT_ERR_DEVICE;
    }
    return WT_OK;
}

}  // extern "C"
