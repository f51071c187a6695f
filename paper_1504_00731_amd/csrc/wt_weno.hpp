// WENO-theta interface reconstruction, FP64 device code for gfx950.
//
// One call reconstructs the value of the numerical flux h at x_{j+1/2} from
// the six split flux values f_{j-2} .. f_{j+3} of the stencil S^6:
//   * four 3-point candidate fluxes, those of S0, S1, S2 (Sec. 2.2) and of the
//     most downwind S3 (Sec. 2.3);
//   * the central smoothness indicators beta~_k (Sec. 3.1), beta~_3 measured
//     on the extended sub-stencil {x_j .. x_{j+3}} in its modified form;
//   * the restriction: all beta~_k become 0 when
//     max_k beta~_k / (eps + min_k beta~_k) <= alpha_R (Sec. 3.1);
//   * tau_5 and tau_6, the indicators of S^5 and S^6, and the switch
//     (tau, theta) = (tau_6, 0) if tau_6 < tau_5 else (tau_5, 1);
//   * gamma^theta (theta = 1: 5th-order upwind weights, theta = 0: 6th-order
//     central weights) and omega_k = alpha_k / sum alpha_l with
//     alpha_k = gamma_k (1 + tau / (eps + beta~_k)) (Sec. 3).
//
// Exactness contract: the file is compiled without floating-point
// contraction and every quantity is formed by the same sequence of IEEE
// double operations (same association, same constants) as the plain
// definition of each formula, so the result is bit-identical to any other
// evaluation of the formulas in that order.  The theta and restriction
// decisions therefore never flip against such a reference.
#pragma once
#pragma clang fp contract(off)

#include <cmath>

#include "wt_common.hpp"
#include "wt_round.hpp"

namespace wt {

// Linear weights gamma^theta_k = (1+theta)/20, 3(3+theta)/20, 3(3-theta)/20,
// (1-theta)/20, folded for the two values theta takes.
struct GammaTheta {
    static constexpr double g0_t0 = (1.0 / 20.0) * (1.0 + 0.0);
    static constexpr double g1_t0 = (3.0 / 20.0) * (3.0 + 0.0);
    static constexpr double g2_t0 = (3.0 / 20.0) * (3.0 - 0.0);
    static constexpr double g3_t0 = (1.0 / 20.0) * (1.0 - 0.0);
    static constexpr double g0_t1 = (1.0 / 20.0) * (1.0 + 1.0);
    static constexpr double g1_t1 = (3.0 / 20.0) * (3.0 + 1.0);
    static constexpr double g2_t1 = (3.0 / 20.0) * (3.0 - 1.0);
    static constexpr double g3_t1 = (1.0 / 20.0) * (1.0 - 1.0);
};

WT_HD double sq(double x) { return x * x; }

// The scheme's constants as the reconstructions take them: eps, alpha_R and
// reps = RN(1 / eps) (formed once on the host, where division is IEEE).
struct WenoConst {
    double eps, alpha_R, reps;
};

// s0..s5 = f_{j-2} .. f_{j+3}.
WT_HD double weno_theta(double s0, double s1, double s2, double s3, double s4, double s5,
                        double eps, double alpha_R, double reps)
{
    // candidate fluxes
    const double q0 = (2.0 / 6.0) * s0 - (7.0 / 6.0) * s1 + (11.0 / 6.0) * s2;
    const double q1 = -(1.0 / 6.0) * s1 + (5.0 / 6.0) * s2 + (2.0 / 6.0) * s3;
    const double q2 = (2.0 / 6.0) * s2 + (5.0 / 6.0) * s3 - (1.0 / 6.0) * s4;
    const double q3 = (11.0 / 6.0) * s3 - (7.0 / 6.0) * s4 + (2.0 / 6.0) * s5;

    // central smoothness indicators
    double b0 = (13.0 / 12.0) * sq(s0 - 2.0 * s1 + s2) + sq(s0 - 3.0 * s1 + 2.0 * s2);
    double b1 = (13.0 / 12.0) * sq(s1 - 2.0 * s2 + s3) + sq(s3 - s2);
    double b2 = (13.0 / 12.0) * sq(s2 - 2.0 * s3 + s4) + sq(s2 - s3);
    double b3 = (13.0 / 48.0) * sq(3.0 * s2 - 7.0 * s3 + 5.0 * s4 - s5) + sq(2.0 * s3 - 3.0 * s4 + s5);

    // restriction (all or none): R = bmax / (eps + bmin) <= alpha_R.  The
    // product test decides it without the quotient unless bmax is within
    // 2^-40 of alpha_R (eps + bmin); RN is monotone, so outside that band the
    // decision equals the one on the rounded quotient.
    // (the indicators are sums of squares, never -0, so for finite data the
    // hardware max/min give exactly the running comparisons of the definition)
    const double bmax = __builtin_fmax(__builtin_fmax(__builtin_fmax(b0, b1), b2), b3);
    const double bmin = __builtin_fmin(__builtin_fmin(__builtin_fmin(b0, b1), b2), b3);
    const double den = eps + bmin;
    const double lim = alpha_R * den;
    bool restricted;
    if (bmax < lim * (1.0 - 0x1p-40)) restricted = true;
    else if (bmax > lim * (1.0 + 0x1p-40)) restricted = false;
    else restricted = div_rn(bmax, den) <= alpha_R;

    // large-stencil indicators and the theta switch
    const double tau5 = (13.0 / 12.0) * sq(s0 - 4.0 * s1 + 6.0 * s2 - 4.0 * s3 + s4) +
                        sq(-s1 + 3.0 * s2 - 3.0 * s3 + s4);
    const double tau6 = (13.0 / 12.0) * sq(-s0 + 5.0 * s1 - 10.0 * s2 + 10.0 * s3 - 5.0 * s4 + s5) +
                        0.25 * sq(s0 - 3.0 * s1 + 2.0 * s2 + 2.0 * s3 - 3.0 * s4 + s5);
    const bool central = tau6 < tau5;           // theta = 0
    const double tau = central ? tau6 : tau5;
    const double g0 = central ? GammaTheta::g0_t0 : GammaTheta::g0_t1;
    const double g1 = central ? GammaTheta::g1_t0 : GammaTheta::g1_t1;
    const double g2 = central ? GammaTheta::g2_t0 : GammaTheta::g2_t1;
    const double g3 = central ? GammaTheta::g3_t0 : GammaTheta::g3_t1;

    // alpha_k = gamma_k (1 + tau / (eps + beta~_k)); restricted indicators are
    // all zero, so the four quotients are one: tau / (eps + 0) = tau / eps,
    // formed from the nearest reciprocal of eps
    double d0, d1, d2, d3;
    if (restricted) {
        d0 = div_by_recip_checked(tau, eps, reps);
        d1 = d0;
        d2 = d0;
        d3 = d0;
    } else {
        d0 = div_rn(tau, eps + b0);
        d1 = div_rn(tau, eps + b1);
        d2 = div_rn(tau, eps + b2);
        d3 = div_rn(tau, eps + b3);
    }
    const double a0 = g0 * (1.0 + d0);
    const double a1 = g1 * (1.0 + d1);
    const double a2 = g2 * (1.0 + d2);
    const double a3 = g3 * (1.0 + d3);
    const double sum = a0 + a1 + a2 + a3;

    // omega_k = alpha_k / sum share the denominator: one reciprocal (sum is at
    // least about 1, since the alpha_k are at least the gamma_k, which sum to 1)
    double w0, w1, w2, w3;
    if (sum <= 0x1p+1000) {
        const double y = recip_rn(sum);
        w0 = div_by_recip(a0, sum, y);
        w1 = div_by_recip(a1, sum, y);
        w2 = div_by_recip(a2, sum, y);
        w3 = div_by_recip(a3, sum, y);
    } else {
        w0 = div_rn(a0, sum);
        w1 = div_rn(a1, sum);
        w2 = div_rn(a2, sum);
        w3 = div_rn(a3, sum);
    }
    return w0 * q0 + w1 * q1 + w2 * q2 + w3 * q3;
}

// ---------------------------------------------------------------------------
// Fast FP64 reconstruction (precision mode WT_FP64_FAST).
//
// The same formulas and decisions, evaluated with fused multiply-adds and
// without correctly rounded quotients:
//   * where the restriction holds every beta~_k is zero, so the four alpha_k
//     share the factor 1 + tau / eps and the weights are exactly gamma^theta:
//     h = sum gamma_k q_k, no quotient at all, which is the 5th-order upwind
//     (theta = 1) or 6th-order central (theta = 0) linear reconstruction, formed
//     from differences the indicators need anyway (fast_linear);
//   * elsewhere alpha_k = gamma_k + gamma_k tau / (eps + beta~_k) from fast
//     reciprocals (hardware estimate and two Newton steps), and
//     h = (sum alpha_k q_k) / (sum alpha_k) by one more.
// The results differ from the plain evaluation by rounding only; the theta and
// restriction decisions can differ only where their two sides are within the
// rounding of the indicators (a legitimate flip).
//
// Every fused multiply-add is written out, in one fixed form, and the compiler
// contracts nothing: a reconstruction is inlined twice per field (the two split
// halves), and the mirror image of an interface hands one copy's stencil, negated,
// to the other.  Copies contracted differently would break the exact mirror
// symmetry of symmetric flows; with a fixed form h(-v) = -h(v) bit for bit.
// ---------------------------------------------------------------------------

// Smoothness indicators and the two theta indicators of a stencil, by fused
// multiply-adds, with the differences they are built from that the linear
// reconstruction reuses.  Everything is formed from six first differences of the
// stencil: each second difference is the sum of two of them, the fourth difference
// of tau5 comes from the second differences, and the second term of tau6 is the sum
// of the second terms of beta~_0 and beta~_3.  (Differences of neighbouring values
// are also the accurate order: they are exact when the values are within a factor of
// two.)
struct FastStencil {
    double b0, b1, b2, b3;     // beta~_k
    double tau5, tau6;
    double d0, d1;             // second differences s_k - 2 s_{k+1} + s_{k+2}, k = 0, 1
    double n2;                 // the negated third one, -(s2 - 2 s3 + s4)
    double d5;                 // fifth difference -s0 + 5 s1 - 10 s2 + 10 s3 - 5 s4 + s5
    double e;                  // s3 - s2
};

WT_HD FastStencil fast_stencil(double s0, double s1, double s2, double s3, double s4, double s5)
{
    FastStencil F;
    const double a = s0 - s1, b = s2 - s1, e = s3 - s2, c = s3 - s4, d = s5 - s4, g = s4 - s1;
    F.e = e;
    F.d0 = a + b;
    F.d1 = e - b;
    F.n2 = e + c;
    const double e2 = e * e;
    const double p0 = __builtin_fma(2.0, b, a);                  // s0 - 3 s1 + 2 s2
    const double p3 = __builtin_fma(2.0, c, d);                  // 2 s3 - 3 s4 + s5
    const double r3 = __builtin_fma(-3.0, e, __builtin_fma(-4.0, c, -d));   // 3 s2 - 7 s3 + 5 s4 - s5
    F.b0 = __builtin_fma((13.0 / 12.0) * F.d0, F.d0, p0 * p0);
    F.b1 = __builtin_fma((13.0 / 12.0) * F.d1, F.d1, e2);
    F.b2 = __builtin_fma((13.0 / 12.0) * F.n2, F.n2, e2);
    F.b3 = __builtin_fma((13.0 / 48.0) * r3, r3, p3 * p3);
    const double t1 = __builtin_fma(-2.0, F.d1, F.d0 - F.n2);   // s0 - 4 s1 + 6 s2 - 4 s3 + s4
    const double t2 = __builtin_fma(-3.0, e, g);                 // -s1 + 3 s2 - 3 s3 + s4
    F.tau5 = __builtin_fma((13.0 / 12.0) * t1, t1, t2 * t2);
    F.d5 = __builtin_fma(10.0, e, __builtin_fma(-5.0, g, s5 - s0));
    const double h = p0 + p3;                                    // s0 - 3 s1 + 2 s2 + 2 s3 - 3 s4 + s5
    F.tau6 = __builtin_fma((13.0 / 12.0) * F.d5, F.d5, (0.25 * h) * h);
    return F;
}

// The reconstruction with the linear weights gamma^theta (the restriction in
// force).  Summed over the candidates, the weights give the 5th-order upwind form
// (theta = 1)  (2 s0 - 13 s1 + 47 s2 + 27 s3 - 3 s4) / 60,  which equals
// (s2 + s3) / 2 + (2 d0 - 9 d1 - 3 d2) / 60, and the 6th-order central form
// (theta = 0)  (s0 - 8 s1 + 37 s2 + 37 s3 - 8 s4 + s5) / 60,  which is the upwind
// one plus d5 / 60.  The differences come from the indicators, so this costs a
// few operations beside them, and a constant stencil gives back its value exactly
// (every difference is zero).
WT_HD double fast_linear(const FastStencil &F, double s2, bool central)
{
    const double corr = __builtin_fma(3.0, F.n2, __builtin_fma(-9.0, F.d1, 2.0 * F.d0));
    const double up = __builtin_fma(1.0 / 60.0, corr, __builtin_fma(0.5, F.e, s2));
    const double ce = __builtin_fma(1.0 / 60.0, F.d5, up);
    return central ? ce : up;
}

// The candidate fluxes q_0 .. q_3 of the four 3-point sub-stencils.
struct FastCandidates {
    double q0, q1, q2, q3;
};

WT_HD FastCandidates fast_candidates(double s0, double s1, double s2, double s3, double s4, double s5)
{
    FastCandidates Q;
    Q.q0 = __builtin_fma(11.0 / 6.0, s2, __builtin_fma(-7.0 / 6.0, s1, (2.0 / 6.0) * s0));
    Q.q1 = __builtin_fma(2.0 / 6.0, s3, __builtin_fma(5.0 / 6.0, s2, (-1.0 / 6.0) * s1));
    Q.q2 = __builtin_fma(-1.0 / 6.0, s4, __builtin_fma(5.0 / 6.0, s3, (2.0 / 6.0) * s2));
    Q.q3 = __builtin_fma(2.0 / 6.0, s5, __builtin_fma(-7.0 / 6.0, s4, (11.0 / 6.0) * s3));
    return Q;
}

WT_HD double weno_theta_fast(double s0, double s1, double s2, double s3, double s4, double s5,
                             double eps, double alpha_R)
{
    const FastStencil F = fast_stencil(s0, s1, s2, s3, s4, s5);
    const double bmax = __builtin_fmax(__builtin_fmax(F.b0, F.b1), __builtin_fmax(F.b2, F.b3));
    const double bmin = __builtin_fmin(__builtin_fmin(F.b0, F.b1), __builtin_fmin(F.b2, F.b3));
    const bool restricted = bmax <= alpha_R * (eps + bmin);
    const bool central = F.tau6 < F.tau5;
    if (restricted) return fast_linear(F, s2, central);
    const FastCandidates Q = fast_candidates(s0, s1, s2, s3, s4, s5);
    const double g0 = central ? GammaTheta::g0_t0 : GammaTheta::g0_t1;
    const double g1 = central ? GammaTheta::g1_t0 : GammaTheta::g1_t1;
    const double g2 = central ? GammaTheta::g2_t0 : GammaTheta::g2_t1;
    const double g3 = central ? GammaTheta::g3_t0 : GammaTheta::g3_t1;
    const double tau = central ? F.tau6 : F.tau5;
    const double a0 = __builtin_fma(g0 * tau, rcp_fast(eps + F.b0), g0);
    const double a1 = __builtin_fma(g1 * tau, rcp_fast(eps + F.b1), g1);
    const double a2 = __builtin_fma(g2 * tau, rcp_fast(eps + F.b2), g2);
    const double a3 = __builtin_fma(g3 * tau, rcp_fast(eps + F.b3), g3);
    const double num = __builtin_fma(a3, Q.q3, __builtin_fma(a2, Q.q2, __builtin_fma(a1, Q.q1, a0 * Q.q0)));
    return num * rcp_fast(a0 + a1 + a2 + a3);
}

// ---------------------------------------------------------------------------
// FP32 weights (precision mode WT_FP32_RECON).
//
// The candidate fluxes, the indicators and both decisions are those of the fast
// FP64 form above (the same fused multiply-adds, so the decisions are FP64
// decisions); where the restriction holds the weights are gamma^theta exactly.
// Elsewhere the quotients tau / (eps + beta~_k) and the weights alpha_k are
// FP32 (eps + beta~_k >= eps keeps them clear of FP32 underflow), and the
// weighted sum and its normalisation are FP64.  The FP32 rounding of the
// weights (about 6e-8 relative) moves the flux by that fraction of the spread
// of the candidate fluxes.
//
// The FP32 reciprocals are refined to nearly always correctly rounded: the
// hardware reciprocal is accurate to one ulp but not unbiased, and a bias that
// moves the weights the same way at every interface accumulates over the time
// steps instead of averaging out.
// ---------------------------------------------------------------------------

// 1/x for normal x > 0: the hardware estimate and one Newton step.
WT_HD float rcp_f32(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    const float r = __builtin_amdgcn_rcpf(x);
    return __builtin_fmaf(r, __builtin_fmaf(-x, r, 1.0f), r);
#else
    return 1.0f / x;
#endif
}

WT_HD double weno_theta_fp32_recon(const double *v, double eps, float alpha_R)
{
    const FastStencil F = fast_stencil(v[0], v[1], v[2], v[3], v[4], v[5]);
    const double bmax = __builtin_fmax(__builtin_fmax(F.b0, F.b1), __builtin_fmax(F.b2, F.b3));
    const double bmin = __builtin_fmin(__builtin_fmin(F.b0, F.b1), __builtin_fmin(F.b2, F.b3));
    const bool restricted = bmax <= (double)alpha_R * (eps + bmin);
    const bool central = F.tau6 < F.tau5;
    if (restricted) return fast_linear(F, v[2], central);
    const FastCandidates Q = fast_candidates(v[0], v[1], v[2], v[3], v[4], v[5]);
    const double g0 = central ? GammaTheta::g0_t0 : GammaTheta::g0_t1;
    const double g1 = central ? GammaTheta::g1_t0 : GammaTheta::g1_t1;
    const double g2 = central ? GammaTheta::g2_t0 : GammaTheta::g2_t1;
    const double g3 = central ? GammaTheta::g3_t0 : GammaTheta::g3_t1;
    // the weights in FP32 (tau is at most about 1e30 for flux values up to 1e14)
    const float tau = (float)__builtin_fmin(central ? F.tau6 : F.tau5, 0x1p+100);
    const float a0 = __builtin_fmaf((float)g0 * tau, rcp_f32((float)__builtin_fmin(eps + F.b0, 0x1p+100)), (float)g0);
    const float a1 = __builtin_fmaf((float)g1 * tau, rcp_f32((float)__builtin_fmin(eps + F.b1, 0x1p+100)), (float)g1);
    const float a2 = __builtin_fmaf((float)g2 * tau, rcp_f32((float)__builtin_fmin(eps + F.b2, 0x1p+100)), (float)g2);
    const float a3 = __builtin_fmaf((float)g3 * tau, rcp_f32((float)__builtin_fmin(eps + F.b3, 0x1p+100)), (float)g3);
    const double w0 = a0, w1 = a1, w2 = a2, w3 = a3;
    const double num = __builtin_fma(w3, Q.q3, __builtin_fma(w2, Q.q2, __builtin_fma(w1, Q.q1, w0 * Q.q0)));
    return num * rcp_fast(w0 + w1 + w2 + w3);
}

}  // namespace wt
