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
//   S.v(k, d)  velocity along axis d;  S.p(k) pressure;  S.sr(k) sqrt(rho);
//   S.H(k) total enthalpy                          (Euler)
//   S.u(k), S.f(k) state and flux value             (scalar)
#pragma once
#pragma clang fp contract(off)

#include "wt_common.hpp"
#include "wt_physics.hpp"
#include "wt_weno.hpp"

namespace wt {

// al[s]: Lax-Friedrichs speed of field s for this direction.  F receives the
// flux in canonical component order.  Returns false if the Roe sound speed is
// not real.
template <int NDIM, int DIR, class Acc>
WT_HD bool euler_interface_flux(const Acc &S, const double *al, double gamma, double eps,
                                double alpha_R, double *F)
{
    constexpr int M = NDIM + 2;
    constexpr int NT = NDIM - 1;
    double velL[NDIM], velR[NDIM];
#pragma unroll
    for (int k = 0; k < NDIM; ++k) {
        velL[k] = S.v(2, k);
        velR[k] = S.v(3, k);
    }
    const RoeBasis<NDIM> B =
        roe_basis<NDIM, DIR>(S.sr(2), velL, S.H(2), S.sr(3), velR, S.H(3), gamma);

    double hs[M];
#pragma unroll
    for (int s = 0; s < M; ++s) {
        const double a = al[s];
        double vp[6], vm[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            // permuted state and normal flux of point k
            const double U0 = S.U(k, 0);
            const double Un = S.U(k, 1 + DIR);
            double Ut[NT > 0 ? NT : 1], vt[NT > 0 ? NT : 1];
#pragma unroll
            for (int q = 0; q < NT; ++q) {
                Ut[q] = S.U(k, 1 + tangential_axis<DIR>(q));
                vt[q] = S.v(k, tangential_axis<DIR>(q));
            }
            const double UE = S.U(k, NDIM + 1);
            const double vn = S.v(k, DIR);
            const double p = S.p(k);
            const double f0 = Un;
            const double f1 = Un * vn + p;
            const double fE = vn * (UE + p);
            double q, w;
            if (s < 3) {
                const double ln0 = s == 0 ? B.l0n0 : (s == 1 ? B.l1n0 : B.l2n0);
                const double ln1 = s == 0 ? B.l0n1 : (s == 1 ? B.l1n1 : B.l2n1);
                const double lE = s == 0 ? B.l0E : (s == 1 ? B.l1E : B.l2E);
                q = ln0 * U0 + ln1 * Un;
                w = ln0 * f0 + ln1 * f1;
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const double lt = s == 0 ? B.l0t[t] : (s == 1 ? B.l1t[t] : B.l2t[t]);
                    q = q + lt * Ut[t];
                    w = w + lt * (Un * vt[t]);
                }
                q = q + lE * UE;
                w = w + lE * fE;
            } else {
                // shear field of tangential direction s - 3: row (-u_t, 0, .., 1, .., 0)
                const int t = s - 3;
                const double nut = -B.ut[t];
                q = nut * U0 + Ut[t];
                w = nut * f0 + Un * vt[t];
            }
            vp[k] = 0.5 * (w + a * q);
            vm[5 - k] = 0.5 * (w - a * q);
        }
        hs[s] = weno_theta(vp[0], vp[1], vp[2], vp[3], vp[4], vp[5], eps, alpha_R) +
                weno_theta(vm[0], vm[1], vm[2], vm[3], vm[4], vm[5], eps, alpha_R);
    }

    // back-projection F = R h: the acoustic pair first, then the entropy
    // field, then the shear fields (a mirrored state gives the mirrored flux)
    const double un = B.un, c = B.c;
    F[0] = (hs[0] + hs[2]) + hs[1];
    F[1 + DIR] = ((un - c) * hs[0] + (un + c) * hs[2]) + un * hs[1];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const double ut = B.ut[t];
        F[1 + tangential_axis<DIR>(t)] = ((ut * hs[0] + ut * hs[2]) + ut * hs[1]) + hs[3 + t];
    }
    double e = (B.H - un * c) * hs[0] + (B.H + un * c) * hs[2];
    e = e + B.q2 * hs[1];
#pragma unroll
    for (int t = 0; t < NT; ++t) e = e + B.ut[t] * hs[3 + t];
    F[M - 1] = e;
    return B.ok;
}

template <class Acc>
WT_HD double scalar_interface_flux(const Acc &S, double al, double eps, double alpha_R)
{
    double vp[6], vm[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const double x = S.u(k), f = S.f(k);
        vp[k] = 0.5 * (f + al * x);
        vm[5 - k] = 0.5 * (f - al * x);
    }
    return weno_theta(vp[0], vp[1], vp[2], vp[3], vp[4], vp[5], eps, alpha_R) +
           weno_theta(vm[0], vm[1], vm[2], vm[3], vm[4], vm[5], eps, alpha_R);
}

}  // namespace wt
