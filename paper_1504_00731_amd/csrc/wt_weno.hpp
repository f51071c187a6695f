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
// FP32 reconstruction (precision mode WT_FP32_RECON).
//
// WENO-theta is invariant under adding a constant to the six values (each
// candidate's coefficients sum to one; the indicators use differences only)
// and, with epsilon scaled by S^2, under scaling them by S.  The FP64 stencil
// is therefore shifted by its point f_j and scaled by an exact power of two
// to magnitude <= 1 before it is rounded to FP32; the reconstruction runs in
// FP32, and the result is scaled back and shifted in FP64.  A constant
// stencil reconstructs to exactly f_j.
//
// Every quotient is (nearly always) correctly rounded: the hardware
// reciprocal is accurate to one ulp but not unbiased, and a bias that scales
// all reconstructed deviations the same way accumulates over the time steps
// instead of averaging out (about 20x the L1 difference to the FP64 path over
// 500 steps of Riemann data, against round-to-nearest quotients).
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

// a / b for normal b > 0 with the reciprocal r = rcp_f32(b): one residual
// correction of the product.
WT_HD float div_f32(float a, float b, float r)
{
#if defined(__HIP_DEVICE_COMPILE__)
    const float q = a * r;
    return __builtin_fmaf(__builtin_fmaf(-b, q, a), r, q);
#else
    (void)r;
    return a / b;
#endif
}

WT_HD float weno_theta_f32(float s0, float s1, float s2, float s3, float s4, float s5, float eps,
                           float alpha_R)
{
#pragma clang fp contract(fast)
    const float q0 = (2.0f / 6.0f) * s0 - (7.0f / 6.0f) * s1 + (11.0f / 6.0f) * s2;
    const float q1 = -(1.0f / 6.0f) * s1 + (5.0f / 6.0f) * s2 + (2.0f / 6.0f) * s3;
    const float q2 = (2.0f / 6.0f) * s2 + (5.0f / 6.0f) * s3 - (1.0f / 6.0f) * s4;
    const float q3 = (11.0f / 6.0f) * s3 - (7.0f / 6.0f) * s4 + (2.0f / 6.0f) * s5;
    float t1, t2;
    t1 = s0 - 2.0f * s1 + s2;
    t2 = s0 - 3.0f * s1 + 2.0f * s2;
    const float b0 = (13.0f / 12.0f) * t1 * t1 + t2 * t2;
    t1 = s1 - 2.0f * s2 + s3;
    t2 = s3 - s2;
    const float b1 = (13.0f / 12.0f) * t1 * t1 + t2 * t2;
    t1 = s2 - 2.0f * s3 + s4;
    t2 = s2 - s3;
    const float b2 = (13.0f / 12.0f) * t1 * t1 + t2 * t2;
    t1 = 3.0f * s2 - 7.0f * s3 + 5.0f * s4 - s5;
    t2 = 2.0f * s3 - 3.0f * s4 + s5;
    const float b3 = (13.0f / 48.0f) * t1 * t1 + t2 * t2;
    const float bmax = fmaxf(fmaxf(b0, b1), fmaxf(b2, b3));
    const float bmin = fminf(fminf(b0, b1), fminf(b2, b3));
    const bool restricted = bmax <= alpha_R * (eps + bmin);
    t1 = s0 - 4.0f * s1 + 6.0f * s2 - 4.0f * s3 + s4;
    t2 = -s1 + 3.0f * s2 - 3.0f * s3 + s4;
    const float tau5 = (13.0f / 12.0f) * t1 * t1 + t2 * t2;
    t1 = -s0 + 5.0f * s1 - 10.0f * s2 + 10.0f * s3 - 5.0f * s4 + s5;
    t2 = s0 - 3.0f * s1 + 2.0f * s2 + 2.0f * s3 - 3.0f * s4 + s5;
    const float tau6 = (13.0f / 12.0f) * t1 * t1 + 0.25f * t2 * t2;
    const bool central = tau6 < tau5;
    const float tau = central ? tau6 : tau5;
    const float g0 = central ? 0.05f : 0.1f;
    const float g1 = central ? 0.45f : 0.6f;
    const float g2 = central ? 0.45f : 0.3f;
    const float g3 = central ? 0.05f : 0.0f;
    // restricted: all indicators are zero and the weights are gamma exactly
    const float a0 = restricted ? g0 : g0 + g0 * tau * rcp_f32(eps + b0);
    const float a1 = restricted ? g1 : g1 + g1 * tau * rcp_f32(eps + b1);
    const float a2 = restricted ? g2 : g2 + g2 * tau * rcp_f32(eps + b2);
    const float a3 = restricted ? g3 : g3 + g3 * tau * rcp_f32(eps + b3);
    const float sum = a0 + a1 + a2 + a3;
    return div_f32(a0 * q0 + a1 * q1 + a2 * q2 + a3 * q3, sum, rcp_f32(sum));
}

// The reconstruction of six FP64 values through the FP32 routine.
WT_HD double weno_theta_fp32_recon(const double *v, double eps, float alpha_R)
{
    const double c = v[2];
    double m = 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const double d = __builtin_fabs(v[k] - c);
        m = d > m ? d : m;
    }
    int e;
    (void)__builtin_frexp(m, &e);               // m < 2^e (e = 0 for m = 0)
    float d[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) d[k] = (float)__builtin_ldexp(v[k] - c, -e);
    double es = __builtin_ldexp(eps, -2 * e);
    es = es < 0x1p-100 ? 0x1p-100 : (es > 0x1p+126 ? 0x1p+126 : es);
    const float h = weno_theta_f32(d[0], d[1], d[2], d[3], d[4], d[5], (float)es, alpha_R);
    return c + __builtin_ldexp((double)h, e);
}

}  // namespace wt
