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
template <int NDIM>
WT_HD bool euler_cell(const double *uc, double gamma, double *vel,
                                           double &p, double &H)
{
    const double rho = uc[0];
    const double E = uc[NDIM + 1];
    const double y = div_rn(1.0, rho);          // shared by the quotients by rho
#pragma unroll
    for (int k = 0; k < NDIM; ++k) vel[k] = div_by_recip(uc[1 + k], rho, y);
    const double v2 = sum_sq_xyz<NDIM>(vel);
    p = (gamma - 1.0) * (E - 0.5 * rho * v2);
    H = div_by_recip(E + p, rho, y);
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
    // left eigenvectors
    double l0n0, l0n1, l0t[2], l0E;    // row 0 (u_n - c)
    double l1n0, l1n1, l1t[2], l1E;    // row 1 (u_n)
    double l2n0, l2n1, l2t[2], l2E;    // row 2 (u_n + c)
    bool ok;
};

template <int NDIM, int DIR>
WT_HD RoeBasis<NDIM> roe_basis(double srL, const double *velL, double HL,
                                                    double srR, const double *velR, double HR,
                                                    double gamma)
{
    RoeBasis<NDIM> B;
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
    B.l0n0 = 0.5 * (b2 + uc);
    B.l0n1 = -0.5 * (b1 * un + ic);
    B.l1n0 = 1.0 - b2;
    B.l1n1 = b1 * un;
    B.l2n0 = 0.5 * (b2 - uc);
    B.l2n1 = -0.5 * (b1 * un - ic);
#pragma unroll
    for (int t = 0; t < NDIM - 1; ++t) {
        B.l0t[t] = -0.5 * (b1 * B.ut[t]);
        B.l1t[t] = b1 * B.ut[t];
        B.l2t[t] = -0.5 * (b1 * B.ut[t]);
    }
    B.l0E = 0.5 * b1;
    B.l1E = -b1;
    B.l2E = 0.5 * b1;
    return B;
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
