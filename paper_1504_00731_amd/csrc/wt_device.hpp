// Device-side building blocks shared by the gfx950 kernels: the device state
// of a context, index maps of the boundary conditions, wave/block max
// reductions into the Lax-Friedrichs speed slots, the wave speeds of a cell,
// and accessors that serve an interface's stencil from a staged LDS tile.
#pragma once
#pragma clang fp contract(off)

#include "wt_bc.hpp"
#include <hip/hip_runtime.h>

#include <cstdint>

#include "wenotheta.h"
#include "wt_flux.hpp"

namespace wt {

constexpr int kThreads = 256;
constexpr int kSlots = 3;        // ring of Lax-Friedrichs speed slots
constexpr int kSlotLen = 16;     // [dir * 5 + field]
constexpr int kXcds = 8;         // accelerator complex dies of an MI355X, one L2 each
constexpr int kErrNonphysical = 1;
constexpr int kErrNonfinite = 2;

struct DevState {
    unsigned long long alpha[kSlots][kSlotLen];  // non-negative doubles as bits
    double dt;
    double t;
    double t_end;
    double tn;            // time at the start of the current step
    long long steps;
    long long max_steps;
    int done;
    int err;
};

// Sweep direction DIR, tile TX x TN with TX * (TN + 1) == kThreads interfaces.

__device__ __forceinline__ double bits_to_double(unsigned long long b)
{
    return __longlong_as_double(static_cast<long long>(b));
}

__device__ __forceinline__ unsigned long long double_to_bits(double d)
{
    return static_cast<unsigned long long>(__double_as_longlong(d));
}

// The hardware maximum of two doubles.  The compiler's maxnum would first quiet the
// operand that comes out of a lane move (it cannot know it to be an arithmetic
// result), one more instruction per step; in IEEE mode v_max_f64 already returns
// the other operand for a quiet NaN.  The two wait states after it cover a DPP move
// that reads the result next (a dependency the compiler does not track through an
// asm statement).
__device__ __forceinline__ double hw_max(double a, double b)
{
    double r;
    __asm__("v_max_f64 %0, %1, %2\n\ts_nop 1" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// One step of a wave reduction of non-negative values by data-parallel primitives:
// every lane takes the maximum of its value and the value DPP control CTRL moves to
// it (both 32-bit halves moved alike).  Every row is written and a lane without a
// source lane reads zero (bound_ctrl), which leaves its maximum unchanged, so the
// move keeps no old value: no copy of the operand before it.
template <int CTRL>
__device__ __forceinline__ double dpp_max_step(double v)
{
    const unsigned long long b = double_to_bits(v);
    const int lo = (int)(unsigned)(b & 0xffffffffull), hi = (int)(unsigned)(b >> 32);
    const int lo2 = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xf, 0xf, true);
    const int hi2 = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xf, 0xf, true);
    const double o = bits_to_double(((unsigned long long)(unsigned)hi2 << 32) | (unsigned)lo2);
    return hw_max(v, o);
}

// Maximum over the wave of non-negative speeds, left in lane 63 (other lanes hold
// partial maxima or values of no use): within quads, half rows and rows by
// permutations, then row 0's maximum into row 1 and row 2's into row 3
// (row_bcast:15), then lane 31's, the maximum of rows 0-1, into rows 2-3
// (row_bcast:31).  Lane 63 only ever combines values of the wave (or zero), whatever
// the broadcasts leave in rows 0-2.  Six VALU steps and no LDS round trips (a
// butterfly of lane shuffles takes six through the LDS crossbar); the hardware max
// returns one of the values, so any order gives the same bits, and a NaN speed,
// which the caller reports as an error anyway, is dropped instead of taken.
__device__ __forceinline__ double wave_max_to_lane63(double v)
{
    v = dpp_max_step<0xb1>(v);      // quad_perm [1,0,3,2]
    v = dpp_max_step<0x4e>(v);      // quad_perm [2,3,0,1]
    v = dpp_max_step<0x141>(v);     // row_half_mirror
    v = dpp_max_step<0x140>(v);     // row_mirror
    v = dpp_max_step<0x142>(v);     // row_bcast:15
    v = dpp_max_step<0x143>(v);     // row_bcast:31
    return v;
}

// Raise slot[k] to v (v >= 0).  A relaxed device-scope read first skips the
// atomic when the slot already holds at least v (values only increase
// between the zeroing and the reading of a slot).
__device__ __forceinline__ void slot_max(unsigned long long *p, double v)
{
    const unsigned long long vb = double_to_bits(v);
    const unsigned long long cur = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (vb > cur) atomicMax(p, vb);
}

// Maximum over each row of 16 lanes of non-negative speeds, in every lane of the
// row: the first four steps of wave_max_to_lane63.
__device__ __forceinline__ double row_max(double v)
{
    v = dpp_max_step<0xb1>(v);      // quad_perm [1,0,3,2]
    v = dpp_max_step<0x4e>(v);      // quad_perm [2,3,0,1]
    v = dpp_max_step<0x141>(v);     // row_half_mirror
    v = dpp_max_step<0x140>(v);     // row_mirror
    return v;
}

// Block-wide max of NV non-negative values per thread, then one slot update per
// slot entry: entry slot_idx[j] takes the block maximum of value src[j] (several
// entries may share a value).  Each wave (ROWS: each row of 16 lanes) reduces its
// values by lane moves and leaves one partial maximum per value in LDS, which the
// slot threads combine.  ROWS saves two lane-move steps per value for a longer
// loop in one wave and four times the partials' LDS, which is for kernels whose
// workgroups per CU the larger table leaves unchanged (the 2D sweeps and the fused
// 2D stage; the 3D sweep and the packed batched pass would lose a workgroup).
template <int NV, int NS, int NT = kThreads, bool ROWS = false>
__device__ __forceinline__ void block_slot_max(double (&v)[NV], unsigned long long *slot,
                                               const int (&src)[NS], const int (&slot_idx)[NS])
{
    constexpr int W = ROWS ? 16 : 64;            // lanes per partial
    constexpr int NR = NT / W;
    __shared__ double red[NV][NR];
    const int lane = threadIdx.x & (W - 1), part = threadIdx.x / W;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double w = ROWS ? row_max(v[k]) : wave_max_to_lane63(v[k]);
        if (lane == W - 1) red[k][part] = w;
    }
    __syncthreads();
    if (threadIdx.x < NS) {
        const int j = threadIdx.x;
        double m = red[src[j]][0];
#pragma unroll
        for (int r = 1; r < NR; ++r) m = __builtin_fmax(m, red[src[j]][r]);
        slot_max(&slot[slot_idx[j]], m);
    }
}

// The hardware maximum of two doubles just read from LDS (no lane move follows, so
// no wait states).
__device__ __forceinline__ double lds_max(double a, double b)
{
    double r;
    __asm__("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// The same block-wide maxima and slot updates as block_slot_max, through LDS
// instead of lane moves, for kernels whose staged tile is free once every cell is
// updated: every thread writes its NV values to the scratch rows (value k of thread
// t at k * NT + t; the first KA values in buffer a, the rest in buffer b), then
// NV x 16 threads each take the maximum of one value over 16 threads 16 apart
// (consecutive threads read consecutive words) into the 16 partials of the value,
// kept in b after its rows (partial g of value k at g * NV + k), and the slot
// threads combine the partials of their value.  It takes no LDS of its own, so the kernel's workgroups per CU are
// unchanged.  Per block this issues about 60 VALU instructions in three waves
// instead of four to six lane-move steps per value in every wave; the maximum
// returns one of its operands, so any order gives the same bits.  The leading
// barrier orders the writes after every read of the tile.
template <int NV, int NS, int NT, int KA>
__device__ __forceinline__ void block_slot_max_lds(const double (&v)[NV], unsigned long long *slot,
                                                   const int (&src)[NS], const int (&slot_idx)[NS],
                                                   double *a, double *b)
{
    constexpr int G = 16;                        // partials per value
    constexpr int R = NT / G;                    // threads per partial
    static_assert(NT % G == 0 && NV * G <= NT && NS <= NT, "one partial per thread");
    double *part = b + (NV - KA) * NT;
    const int t = threadIdx.x;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) (k < KA ? a + k * NT : b + (k - KA) * NT)[t] = v[k];
    __syncthreads();
    if (t < NV * G) {
        const int k = t / G, g = t - k * G;
        const double *row = k < KA ? a + k * NT : b + (k - KA) * NT;
        double m = row[g];
#pragma unroll
        for (int r = 1; r < R; ++r) m = lds_max(m, row[r * G + g]);
        part[g * NV + k] = m;
    }
    __syncthreads();
    if (t < NS) {
        // partials value-fastest: the slot threads read neighbouring words
        const double *p = part + src[t];
        double m = p[0];
#pragma unroll
        for (int g = 1; g < G; ++g) m = lds_max(m, p[g * NV]);
        slot_max(&slot[slot_idx[t]], m);
    }
}

// Wave speeds of one cell (canonical state): per direction |u_d - c|, |u_d|,
// |u_d + c|, with c = sqrt(gamma p / rho).  Returns an error bit mask.
template <int NDIM, bool FAST = false>
__device__ __forceinline__ int euler_speeds(const double *uc, double gamma, double *lam)
{
    double vel[NDIM], p, H;
    const bool ok = euler_cell<NDIM, FAST>(uc, gamma, vel, p, H);
    double c;
    if constexpr (FAST) {
        const double r = rsq_fast(uc[0]);       // the one euler_cell formed 1/rho from
        c = sqrt_fast(gamma * p * (r * r));
    }
    else c = sqrt_rn(div_rn(gamma * p, uc[0]));
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
        lam[3 * d + 0] = __builtin_fabs(vel[d] - c);
        lam[3 * d + 1] = __builtin_fabs(vel[d]);
        lam[3 * d + 2] = __builtin_fabs(vel[d] + c);
    }
    if (ok) return 0;
    bool finite = true;
#pragma unroll
    for (int k = 0; k < NDIM + 2; ++k) finite = finite && __builtin_isfinite(uc[k]);
    return finite ? kErrNonphysical : kErrNonfinite;
}

// Flux-difference quotient of a cell, (F_{i+1/2} - F_{i-1/2}) / dx: correctly
// rounded, or (fast forms) the product with the reciprocal of dx.
template <bool FAST>
WT_HD double flux_quotient(double dF, double dx, double rdx)
{
    if constexpr (FAST) return dF * rdx;
    else return div_by_recip(dF, dx, rdx);
}

// One component of a TVD Runge-Kutta stage (Sec. 2.1): stage 1 u + dt L, stage 2
// 3/4 u^n + 1/4 u^(1) + dt/4 L, stage 3 1/3 u^n + 2/3 u^(2) + 2 dt/3 L, from the
// stage's input uin and u^n (u0, unused in stage 1).  The fast forms use fused
// multiply-adds in one fixed form for every component (the symmetries of a flow
// exchange components).
template <bool FAST>
WT_HD double rk3_stage(int stage, double uin, double L, double dt, double u0)
{
    if constexpr (FAST) {
        const double c1 = stage == 1 ? 1.0 : (stage == 2 ? 0.25 : 2.0 / 3.0);
        const double cdt = (stage == 1 ? 1.0 : (stage == 2 ? 0.25 : 2.0 / 3.0)) * dt;
        const double base = __builtin_fma(cdt, L, c1 * uin);
        if (stage == 1) return base;
        return __builtin_fma(stage == 2 ? 0.75 : 1.0 / 3.0, u0, base);
    } else {
        if (stage == 1) return uin + dt * L;
        if (stage == 2) return 0.75 * u0 + 0.25 * uin + (0.25 * dt) * L;
        return (1.0 / 3.0) * u0 + (2.0 / 3.0) * uin + ((2.0 / 3.0) * dt) * L;
    }
}

// u^n of one cell for a Runge-Kutta stage (components `stride` apart), every
// component read under one branch, so the loads are in flight together instead of
// each waiting in turn; stage 1 reads nothing.
template <int M>
WT_HD void stage_u0(int stage, const double *u0, int64_t stride, int64_t idx, double (&v)[M])
{
    if (stage != 1) {
#pragma unroll
        for (int c = 0; c < M; ++c) v[c] = u0[c * stride + idx];
    } else {
#pragma unroll
        for (int c = 0; c < M; ++c) v[c] = 0.0;
    }
}

// Lax-Friedrichs speeds: per direction d the distinct values |u_d - c|,
// |u_d|, |u_d + c| (value 3 d + s, the order of euler_speeds), reduced once
// each; slot entry d * 5 + s of field s takes value 3 d + s for s = 0, 1, 2
// and 3 d + 1 for the shear fields (NS entries in all).
template <int SYS, int NDIM>
struct SpeedLayout {
    static constexpr int M = Ncomp<SYS, NDIM>::value;
    static constexpr int NV = SYS == SYS_EULER ? 3 * NDIM : 1;
    static constexpr int NS = SYS == SYS_EULER ? NDIM * M : 1;
    __device__ static constexpr int slot_index(int j) { return SYS == SYS_EULER ? (j / M) * 5 + j % M : 0; }
    __device__ static constexpr int value_of_slot(int j)
    {
        return SYS == SYS_EULER ? 3 * (j / M) + (j % M < 3 ? j % M : 1) : 0;
    }
};

// Stencil accessors over the staged tile: point k of the interface owned by
// thread t is tile entry t + k * TX.  With P the tile also holds each point's
// pressure, from which the fast forms project the normal flux (kPressure).
template <int M, int NDIM, int NC, int TX, bool P = false>
struct LdsStencil {
    const double (*u)[NC];
    const double (*fn)[NC];
    const double (*vel)[NC];
    const double *sq, *hh;
    int t;
    const double *pp = nullptr;                 // pressures, where P
    static constexpr bool kPressure = P;
    __device__ double U(int k, int c) const { return u[c][t + k * TX]; }
    __device__ double f(int k, int c) const { return fn[c][t + k * TX]; }
    __device__ double p(int k) const { return pp[t + k * TX]; }
    __device__ double v(int k, int d) const { return vel[d][t + k * TX]; }
    __device__ double sr(int k) const { return sq[t + k * TX]; }
    __device__ double H(int k) const { return hh[t + k * TX]; }
};

// Lax-Friedrichs speed of field s of the sweep direction, from a slot.
// Speeds of the sweep direction read from a slot (per-field maxima), paired
// for the acoustic fields behind reflective walls.
struct SlotSpeeds {
    const unsigned long long *slot;
    int dir;
    bool walls;
    __device__ double raw(int s) const { return bits_to_double(slot[dir * 5 + s]); }
    __device__ double operator()(int s) const
    {
        return split_speed([this](int k) { return raw(k); }, s, walls);
    }
};

// Lax-Friedrichs speeds of one direction's fields staged in LDS (a[s] for field s):
// every lane reads the same word, a broadcast, instead of each field of each
// interface waiting on a device-memory read.
struct LdsSpeeds {
    const double *a;
    __device__ double operator()(int s) const { return a[s]; }
};

template <int NC, int TX>
struct LdsScalarStencil {
    const double *uu, *ff;
    int t;
    __device__ double u(int k) const { return uu[t + k * TX]; }
    __device__ double f(int k) const { return ff[t + k * TX]; }
};

}  // namespace wt
