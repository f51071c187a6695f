// Physics of the supported systems in FP64 for the gfx950 kernels: the
// scalar fluxes, Euler primitives, the Roe mean state and its eigenvectors.
//
// Same exactness contract as wt_weno.hpp: no contraction, and every value is
// formed by one fixed sequence of IEEE operations.
//
// Directions.  A sweep along direction DIR sees the Euler state in the
// permuted component order (rho, m_n, m_t1, [m_t2,] E): the normal momentum
// m_n = m_DIR first, tangential momenta in increasing axis order.  All
// directions run the same code on that order, which is what keeps a state
// that is symmetric under x <-> y exactly symmetric.  Kinetic-energy sums
// always run over the axes in the order x, y, z.
#pragma once
#pragma clang fp contract(off)

#include "wt_common.hpp"
#include "wt_round.hpp"

namespace wt {

enum : int { SYS_LINEAR = 0, SYS_BURGERS = 1, SYS_EULER = 2 };

template <int SYS, int NDIM>
struct Ncomp {
    static constexpr int value = SYS == SYS_EULER ? NDIM + 2 : 1;
};

// Index of the k-th tangential axis of direction DIR (increasing axis order).
template <int DIR>
WT_HD constexpr int tangential_axis(int k)
{
    return k < DIR ? k : k + 1;
}

// Sum of squares over the axes in the order x, y, z.
template <int NDIM>
WT_HD double sum_sq_xyz(const double *v)
{
    double s = v[0] * v[0];
    if constexpr (NDIM > 1) s = s + v[1] * v[1];
    if constexpr (NDIM > 2) s = s + v[2] * v[2];
    return s;
}

// Cell quantities of an Euler state (canonical order rho, m_x.., E):
// velocities, pressure p = (gamma-1)(E - rho |v|^2 / 2) and total enthalpy
// H = (E + p) / rho (Sec. 4.2; the 2D form of Sec. 4.3 with the density
// restored).  Returns false for a non-physical or non-finite state.
// FAST (the fast FP64 and FP32-weight modes): the same quantities with 1/rho formed
// as the square of the refined reciprocal square root (which the staged sqrt(rho)
// shares) and products by it.
template <int NDIM, bool FAST = false>
WT_HD bool euler_cell(const double *uc, double gamma, double *vel,
                                           double &p, double &H)
{
    const double rho = uc[0];
    const double E = uc[NDIM + 1];
    if constexpr (FAST) {
        // no contraction: a fused |v|^2 would round the axes differently, and a state with
        // its velocity components exchanged would no longer give the same pressure
        const double r = rsq_fast(rho);
        const double y = r * r;
#pragma unroll
        for (int k = 0; k < NDIM; ++k) vel[k] = uc[1 + k] * y;
        const double v2 = sum_sq_xyz<NDIM>(vel);
        p = (gamma - 1.0) * (E - 0.5 * rho * v2);
        H = (E + p) * y;
    } else {
        const double y = div_rn(1.0, rho);      // shared by the quotients by rho
#pragma unroll
        for (int k = 0; k < NDIM; ++k) vel[k] = div_by_recip(uc[1 + k], rho, y);
        const double v2 = sum_sq_xyz<NDIM>(vel);
        p = (gamma - 1.0) * (E - 0.5 * rho * v2);
        H = div_by_recip(E + p, rho, y);
    }
    return rho > 0.0 && p > 0.0 && H == H && __builtin_fabs(H) < __builtin_huge_val();
}

// Roe mean state between two cells and the eigen-system of the Roe matrix in
// the permuted order of direction DIR.  Field order: u_n - c, u_n, u_n + c,
// then one shear field per tangential direction.  Only the non-zero entries
// of L and R are kept; the zero entries contribute exact zeros to every
// product in which they appear.
template <int NDIM>
struct RoeBasis {
    double un;                 // normal Roe velocity
    double ut[2];              // tangential Roe velocities
    double c;                  // Roe sound speed
    double H;                  // Roe total enthalpy
    // left eigenvectors, formed row by row from these (left_row)
    double b1;                 // (gamma - 1) / c^2
    double b2;                 // b1 |v~|^2 / 2
    double uc;                 // u_n / c
    double ic;                 // 1 / c
    bool ok;
};

template <int NDIM, int DIR, bool FAST = false>
WT_HD RoeBasis<NDIM> roe_basis(double srL, const double *velL, double HL,
                                                    double srR, const double *velR, double HR,
                                                    double gamma)
{
    RoeBasis<NDIM> B;
    if constexpr (FAST) {
        // fast reciprocals and roots, but no contraction: a fused srL vL + srR vR
        // would round the two sides differently, and the mirror image of an interface
        // (left and right exchanged) would no longer give the mirrored flux bit for bit
        const double yd = rcp_fast(srL + srR);
        double vt[3];
#pragma unroll
        for (int k = 0; k < NDIM; ++k) vt[k] = (srL * velL[k] + srR * velR[k]) * yd;
        const double H = (srL * HL + srR * HR) * yd;
        const double q2 = 0.5 * sum_sq_xyz<NDIM>(vt);
        const double c2 = (gamma - 1.0) * (H - q2);
        B.ok = c2 > 0.0;
        const double ic = rsq_fast(c2);          // 1/c, and c from it
        const double c = c2 * ic;
#pragma unroll
        for (int t = 0; t < NDIM - 1; ++t) B.ut[t] = vt[tangential_axis<DIR>(t)];
        B.un = vt[DIR];
        B.c = c;
        B.H = H;
        B.b1 = (gamma - 1.0) * (ic * ic);
        B.b2 = B.b1 * q2;
        B.uc = B.un * ic;
        B.ic = ic;
        return B;
    }
    const double den = srL + srR;
    const double yd = div_rn(1.0, den);         // shared by the Roe averages
    double vt[3];
#pragma unroll
    for (int k = 0; k < NDIM; ++k) vt[k] = div_by_recip(srL * velL[k] + srR * velR[k], den, yd);
    const double H = div_by_recip(srL * HL + srR * HR, den, yd);
    const double q2 = 0.5 * sum_sq_xyz<NDIM>(vt);
    const double c2 = (gamma - 1.0) * (H - q2);
    B.ok = c2 > 0.0;
    const double c = sqrt_rn(c2);
    const double un = vt[DIR];
#pragma unroll
    for (int t = 0; t < NDIM - 1; ++t) B.ut[t] = vt[tangential_axis<DIR>(t)];
    const double b1 = div_rn(gamma - 1.0, c2);
    const double b2 = b1 * q2;
    const double ic = div_rn(1.0, c);
    const double uc = div_by_recip(un, c, ic);
    B.un = un;
    B.c = c;
    B.H = H;
    B.b1 = b1;
    B.b2 = b2;
    B.uc = uc;
    B.ic = ic;
    return B;
}

// With FRESH, a value the compiler must treat as new here: the expressions
// formed from it stay where they are written instead of being hoisted out of
// the field loop, where they would all be live at once (and, in 3D and in the
// fast and FP32-weight forms, cost a wave per SIMD or spill).  Without FRESH the
// compiler may keep them across the loop, which the plain FP64 1D and 2D sweeps
// can afford.
template <bool FRESH>
WT_HD double opaque(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (FRESH) __asm__ volatile("" : "+v"(x));
#endif
    return x;
}

// The basis values as values the compiler must treat as new at this point (once per
// field, at the top of the field loop): the rows of L and columns of R formed from
// them then stay where they are written instead of being hoisted out of the loop,
// where they would all be live at once.  The values are updated in place, so, unlike
// passing each use through opaque(), no copies are needed to keep the originals.
template <int NDIM>
WT_HD void refresh_basis(RoeBasis<NDIM> &B)
{
#if defined(__HIP_DEVICE_COMPILE__)
    __asm__ volatile("" : "+v"(B.un), "+v"(B.c), "+v"(B.H), "+v"(B.b1), "+v"(B.b2), "+v"(B.uc),
                          "+v"(B.ic));
#pragma unroll
    for (int t = 0; t < NDIM - 1; ++t) __asm__ volatile("" : "+v"(B.ut[t]));
#endif
}

// Row s (0: u_n - c, 1: u_n, 2: u_n + c) of the left eigenvectors in permuted
// order: coefficients of rho, m_n, the tangential momenta and E.
template <int NDIM, bool FRESH>
WT_HD void left_row(const RoeBasis<NDIM> &B, int s, double &ln0, double &ln1, double *lt, double &lE)
{
    const double b1 = opaque<FRESH>(B.b1), b2 = opaque<FRESH>(B.b2), un = opaque<FRESH>(B.un);
    if (s == 0) {
        ln0 = 0.5 * (b2 + opaque<FRESH>(B.uc));
        ln1 = -0.5 * (b1 * un + opaque<FRESH>(B.ic));
#pragma unroll
        for (int t = 0; t < NDIM - 1; ++t) lt[t] = -0.5 * (b1 * opaque<FRESH>(B.ut[t]));
        lE = 0.5 * b1;
    } else if (s == 1) {
        ln0 = 1.0 - b2;
        ln1 = b1 * un;
#pragma unroll
        for (int t = 0; t < NDIM - 1; ++t) lt[t] = b1 * opaque<FRESH>(B.ut[t]);
        lE = -b1;
    } else {
        ln0 = 0.5 * (b2 - opaque<FRESH>(B.uc));
        ln1 = -0.5 * (b1 * un - opaque<FRESH>(B.ic));
#pragma unroll
        for (int t = 0; t < NDIM - 1; ++t) lt[t] = -0.5 * (b1 * opaque<FRESH>(B.ut[t]));
        lE = 0.5 * b1;
    }
}

// Half of row s of the left eigenvectors (fast forms): the split values are
// (w +- a q) / 2, and projecting on the halved row gives w / 2 and q / 2 directly.
// Halving is exact, so every product and sum below is the half of the one formed
// from the full row (outside the subnormal range).
template <int NDIM, bool FRESH>
WT_HD void left_row_half(const RoeBasis<NDIM> &B, int s, double &ln0, double &ln1, double *lt, double &lE)
{
    const double b1 = opaque<FRESH>(B.b1), b2 = opaque<FRESH>(B.b2), un = opaque<FRESH>(B.un);
    if (s == 0) {
        ln0 = 0.25 * (b2 + opaque<FRESH>(B.uc));
        ln1 = -0.25 * (b1 * un + opaque<FRESH>(B.ic));
#pragma unroll
        for (int t = 0; t < NDIM - 1; ++t) lt[t] = -0.25 * (b1 * opaque<FRESH>(B.ut[t]));
        lE = 0.25 * b1;
    } else if (s == 1) {
        const double hb1 = 0.5 * b1;
        ln0 = __builtin_fma(-0.5, b2, 0.5);
        ln1 = hb1 * un;
#pragma unroll
        for (int t = 0; t < NDIM - 1; ++t) lt[t] = hb1 * opaque<FRESH>(B.ut[t]);
        lE = -hb1;
    } else {
        ln0 = 0.25 * (b2 - opaque<FRESH>(B.uc));
        ln1 = -0.25 * (b1 * un - opaque<FRESH>(B.ic));
#pragma unroll
        for (int t = 0; t < NDIM - 1; ++t) lt[t] = -0.25 * (b1 * opaque<FRESH>(B.ut[t]));
        lE = 0.25 * b1;
    }
}

// |v~|^2 / 2 of a Roe basis, recomputed from its velocities in canonical order
// with the operations of roe_basis (so the same value) where the entropy
// column of R needs it.  The velocities first pass through an empty asm, so
// the compiler recomputes the value instead of keeping the one of roe_basis
// alive across the whole field loop (which cost the 2D stage-finishing sweep
// a register spill at 4 waves per SIMD).
template <int NDIM, int DIR>
WT_HD double roe_q2(const RoeBasis<NDIM> &B)
{
    double vt[3];
    vt[DIR] = B.un;
#pragma unroll
    for (int t = 0; t < NDIM - 1; ++t) vt[tangential_axis<DIR>(t)] = B.ut[t];
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
    for (int k = 0; k < NDIM; ++k) __asm__ volatile("" : "+v"(vt[k]));
#endif
    return 0.5 * sum_sq_xyz<NDIM>(vt);
}

}  // namespace wt
