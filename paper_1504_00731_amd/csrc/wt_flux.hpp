// Numerical flux at one interface x_{j+1/2}, FP64, from the six stencil points
// j-2 .. j+3 of its sweep direction.
//
// Euler (Sec. 4.2): Roe mean state of points j and j+1, projection of the
// stencil's conserved states and normal fluxes onto the characteristic fields
// (q = L u, w = L f), global Lax-Friedrichs split v+- = (w +- alpha_s q)/2 per
// field (remark on flux splitting), WENO-theta on v+ over j-2..j+3 and on v-
// over the mirrored stencil j+3..j-2, sum, and back-projection F = R h.
// Scalar: the same split on the flux values, without projection.
//
// The stencil is read through an accessor, so the kernels can serve it from
// LDS and a host build can serve it from arrays:
//   S.U(k, c)  conserved component c (canonical order) of point k = 0..5
//   S.f(k, c)  normal flux component c (canonical order) of point k (plain FP64)
//   S.p(k)     pressure of point k (fast and FP32-weight forms, kPressure)
//   S.v(k, d)  velocity along axis d;  S.sr(k) sqrt(rho);  S.H(k) enthalpy
//   S.u(k), S.f(k) state and flux value            (scalar)
//
// Register use.  The characteristic fields are visited by a loop the
// compiler keeps rolled (the trip count is the same for every lane, so the
// branches on the field index are uniform).  This keeps the live set to one
// field's 12 split values plus the Roe basis and the flux accumulators,
// instead of all fields at once.  The two reconstructions of a field (split
// signs) are independent and are unrolled side by side, so the long division
// chains of one overlap the other's.
#pragma once
#pragma clang fp contract(off)

#include "wt_common.hpp"
#include "wt_physics.hpp"
#include "wt_weno.hpp"

namespace wt {

// One interface reconstruction of six split values in precision mode PREC
// (0: FP64 with the plain operation order, 1: FP32 reconstruction, 2: fast FP64).
template <int PREC>
WT_HD double reconstruct(const double *v, const WenoConst &W)
{
    if constexpr (PREC == 0)
        return weno_theta(v[0], v[1], v[2], v[3], v[4], v[5], W.eps, W.alpha_R, W.reps);
    else if constexpr (PREC == 2)
        return weno_theta_fast(v[0], v[1], v[2], v[3], v[4], v[5], W.eps, W.alpha_R);
    else
        return weno_theta_fp32_recon(v, W.eps, (float)W.alpha_R);
}

// Precision modes 1 (WT_FP32_RECON) and 2 (WT_FP64_FAST) evaluate the FP64 parts of
// an interface (cell quantities, Roe basis, projection, split) with fused
// multiply-adds and fast reciprocals; mode 0 keeps the plain operation order.
template <int PREC>
constexpr bool fast_math()
{
    return PREC != 0;
}

// Normal flux of a cell in canonical component order for direction DIR:
// (rho u_n, rho u_x u_n + p delta_{x,n}, .., u_n (E + p)), formed as
// m_n, m_n u_n + p, m_n u_t, u_n (E + p).
template <int NDIM, int DIR>
WT_HD void euler_normal_flux(const double *uc, const double *vel, double p, double *f)
{
    const double mn = uc[1 + DIR];
    const double un = vel[DIR];
    f[0] = mn;
#pragma unroll
    for (int d = 0; d < NDIM; ++d) f[1 + d] = d == DIR ? mn * un + p : mn * vel[d];
    f[NDIM + 1] = un * (uc[NDIM + 1] + p);
}

// Whether the sweeps of this form recompute the rows of L and columns of R per
// field (opaque<true>) instead of letting the compiler keep them across the
// field loop: the fast and FP32-weight forms and 3D, whose occupancy the saved
// registers raise (the fast 2D x-sweep fits 94 VGPRs and runs 5 waves per SIMD
// instead of 4; the recomputed rows cost about what selecting kept ones did, and
// the 2D Euler 4096^2 step ran 7% faster).  The plain FP64 1D and 2D sweeps keep
// them.
template <int NDIM, int PREC>
constexpr bool fresh_rows()
{
    return PREC != 0 || NDIM == 3;
}

// Characteristic field s of an interface (0: u_n - c, 1: u_n, 2: u_n + c, 3..:
// shear): the stencil projected onto row s of L (q = L u, w = L f), split with the
// field's Lax-Friedrichs speed a = al(s), v+- = (w +- a q) / 2, and reconstructed,
// sign +1 on j-2..j+3 and sign -1 on the mirrored stencil; returns h+ + h-.
template <int NDIM, int DIR, int PREC, bool FRESH, class Acc, class Alpha>
WT_HD double euler_field_flux(const Acc &S, const RoeBasis<NDIM> &B, int s, const Alpha &al,
                              const WenoConst &W)
{
    constexpr int NT = NDIM - 1;
    WT_RELOAD();                                // stencil values come from memory per field
    // row s of L in permuted order
    double ln0, ln1, lE, lt[NT > 0 ? NT : 1];
    int shear = -1;
    if (s < 3) {
        if constexpr (fast_math<PREC>()) left_row_half<NDIM, FRESH>(B, s, ln0, ln1, lt, lE);
        else left_row<NDIM, FRESH>(B, s, ln0, ln1, lt, lE);
    } else {
        shear = s - 3;
        ln0 = -(shear == 0 ? B.ut[0] : B.ut[NT > 1 ? 1 : 0]); ln1 = 0.0; lE = 0.0;
#pragma unroll
        for (int t = 0; t < NT; ++t) lt[t] = 0.0;
    }
    const double a = al(s);
    double vp[6], vm[6];
    if constexpr (fast_math<PREC>()) {
        // fused multiply-adds written out, in one fixed form: the mirror image of an
        // interface (its acoustic fields exchanged, the normal components negated) then
        // forms exactly the negated split values, which a contraction left to the
        // compiler does not guarantee (it may fuse either product of a sum)
        // (the acoustic and entropy rows are halved, so qq and ww are q / 2 and w / 2).
        // The normal flux is not read: it is f = u_n U + p (0, e_n, u_n), so
        // l.f = u_n (l.U) + p (l_n + l_E u_n), three operations from qq instead of a
        // second dot product, and u_n and p instead of the flux components from LDS.
        static_assert(Acc::kPressure, "the fast forms read the points' pressures");
        const double ha = 0.5 * a;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            if (shear < 0) {
                double qq = __builtin_fma(ln1, S.U(k, 1 + DIR), ln0 * S.U(k, 0));
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    qq = __builtin_fma(lt[t], S.U(k, 1 + tangential_axis<DIR>(t)), qq);
                qq = __builtin_fma(lE, S.U(k, NDIM + 1), qq);
                const double un = S.v(k, DIR);
                const double ww = __builtin_fma(un, qq, S.p(k) * __builtin_fma(lE, un, ln1));
                vp[k] = __builtin_fma(a, qq, ww);
                vm[5 - k] = __builtin_fma(-a, qq, ww);
            } else {
                // shear row (-u_t, 0, .., 1, .., 0): l_n = l_E = 0, so l.f = u_n (l.U)
                const int ax = 1 + (shear == 0 ? tangential_axis<DIR>(0) : tangential_axis<DIR>(NT - 1));
                const double qq = __builtin_fma(ln0, S.U(k, 0), S.U(k, ax));
                const double hw = (0.5 * S.v(k, DIR)) * qq;
                vp[k] = __builtin_fma(ha, qq, hw);
                vm[5 - k] = __builtin_fma(-ha, qq, hw);
            }
        }
    } else {
    double w[6], q[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        if (shear < 0) {
            double qq = ln0 * S.U(k, 0) + ln1 * S.U(k, 1 + DIR);
            double ww = ln0 * S.f(k, 0) + ln1 * S.f(k, 1 + DIR);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                qq = qq + lt[t] * S.U(k, 1 + tangential_axis<DIR>(t));
                ww = ww + lt[t] * S.f(k, 1 + tangential_axis<DIR>(t));
            }
            q[k] = qq + lE * S.U(k, NDIM + 1);
            w[k] = ww + lE * S.f(k, NDIM + 1);
        } else {
            // shear row (-u_t, 0, .., 1, .., 0): only two non-zero entries
            const int ax = 1 + (shear == 0 ? tangential_axis<DIR>(0) : tangential_axis<DIR>(NT - 1));
            q[k] = ln0 * S.U(k, 0) + S.U(k, ax);
            w[k] = ln0 * S.f(k, 0) + S.f(k, ax);
        }
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const double aq = a * q[k];
        vp[k] = 0.5 * (w[k] + aq);
        vm[5 - k] = 0.5 * (w[k] - aq);
    }
    }
    double h = 0.0;
#pragma unroll
    for (int sg = 0; sg < 2; ++sg) {
        double v[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) v[k] = sg == 0 ? vp[k] : vm[k];
        const double r = reconstruct<PREC>(v, W);
        h = sg == 0 ? r : h + r;
    }
    return h;
}

// Field visiting order of the back-projection: 0, 2, 1, 3, 4, so that every
// component sums R h as (R_0 h_0 + R_2 h_2) + R_1 h_1 + R_3 h_3 + R_4 h_4.
WT_HD constexpr int field_order(int it)
{
    return it == 1 ? 2 : (it == 2 ? 1 : it);
}

// Add column s of R times h_s to the accumulators (permuted order rho, m_n,
// m_t.., E); the first field in field_order initialises them.
template <int NDIM, int DIR, bool FRESH>
WT_HD void backproject_field(const RoeBasis<NDIM> &B, int s, double h, double *acc)
{
    constexpr int M = NDIM + 2, NT = NDIM - 1;
    const double un = opaque<FRESH>(B.un), c = opaque<FRESH>(B.c);
    if (s == 0) {
        acc[0] = h;
        acc[1] = (un - c) * h;
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[2 + t] = B.ut[t] * h;
        acc[M - 1] = (B.H - un * c) * h;
    } else if (s == 2) {
        acc[0] = acc[0] + h;
        acc[1] = acc[1] + (un + c) * h;
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[2 + t] = acc[2 + t] + B.ut[t] * h;
        acc[M - 1] = acc[M - 1] + (B.H + un * c) * h;
    } else if (s == 1) {
        acc[0] = acc[0] + h;
        acc[1] = acc[1] + un * h;
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[2 + t] = acc[2 + t] + B.ut[t] * h;
        acc[M - 1] = acc[M - 1] + roe_q2<NDIM, DIR>(B) * h;
    } else {
        const int shear = s - 3;
#pragma unroll
        for (int t = 0; t < NT; ++t)
            if (t == shear) acc[2 + t] = acc[2 + t] + h;
        acc[M - 1] = acc[M - 1] + (shear == 0 ? B.ut[0] : B.ut[NT > 1 ? 1 : 0]) * h;
    }
}

// The accumulators in canonical component order.
template <int NDIM, int DIR>
WT_HD void store_interface_flux(const double *acc, double *F)
{
    constexpr int M = NDIM + 2, NT = NDIM - 1;
    F[0] = acc[0];
    F[1 + DIR] = acc[1];
#pragma unroll
    for (int t = 0; t < NT; ++t) F[1 + tangential_axis<DIR>(t)] = acc[2 + t];
    F[M - 1] = acc[M - 1];
}

// Roe basis of the interface between stencil points 2 and 3.
template <int NDIM, int DIR, bool FAST = false, class Acc>
WT_HD RoeBasis<NDIM> interface_basis(const Acc &S, double gamma)
{
    double velL[NDIM], velR[NDIM];
#pragma unroll
    for (int k = 0; k < NDIM; ++k) {
        velL[k] = S.v(2, k);
        velR[k] = S.v(3, k);
    }
    return roe_basis<NDIM, DIR, FAST>(S.sr(2), velL, S.H(2), S.sr(3), velR, S.H(3), gamma);
}

// al(s): Lax-Friedrichs speed of field s for this direction.  F receives the
// flux in canonical component order.  Returns false if the Roe sound speed is
// not real.  FRESH: rows of L and columns of R recomputed per field.
template <int NDIM, int DIR, int PREC, bool FRESH = fresh_rows<NDIM, PREC>(), class Acc, class Alpha>
WT_HD bool euler_interface_flux(const Acc &S, const Alpha &al, double gamma, const WenoConst &W,
                                double *F)
{
    constexpr int M = NDIM + 2;
    RoeBasis<NDIM> B = interface_basis<NDIM, DIR, fast_math<PREC>()>(S, gamma);
    double acc[M];
#pragma unroll 1
    for (int it = 0; it < M; ++it) {
        if constexpr (FRESH) refresh_basis(B);    // rows and columns formed per field
        const int s = field_order(it);
        const double h = euler_field_flux<NDIM, DIR, PREC, false>(S, B, s, al, W);
        backproject_field<NDIM, DIR, false>(B, s, h, acc);
    }
    store_interface_flux<NDIM, DIR>(acc, F);
    return B.ok;
}

template <int PREC, class Acc>
WT_HD double scalar_interface_flux(const Acc &S, double al, const WenoConst &W)
{
    double vp[6], vm[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const double x = S.u(k), f = S.f(k);
        vp[k] = 0.5 * (f + al * x);
        vm[5 - k] = 0.5 * (f - al * x);
    }
    return reconstruct<PREC>(vp, W) + reconstruct<PREC>(vm, W);
}

}  // namespace wt
