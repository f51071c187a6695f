// Correctly rounded FP64 division and square root on gfx950.
//
// The compiler's FP64 division sequence (scale, reciprocal, two Newton steps,
// fused correction) returns a faithful quotient, but not always the nearest
// one: when the exact quotient lies within about 2^-53 ulp of a rounding
// midpoint it can round the wrong way (e.g. 0x1.6666666666663p-2 /
// 0x1.ffffffffffffbp-4).  Every value the kernels produce must be the one a
// plain IEEE evaluation produces, so each quotient and root is finished here
// with an exact test against its neighbour:
//   division (denominator b > 0, q faithful): the remainders r = a - q b and
//     r' = a - q' b of q and of its neighbour q' on the side of a/b are exact
//     (FMA); |r| and |r'| are b times the two distances to a/b, so the
//     smaller one names the nearest double (an exact quotient is never a
//     midpoint);
//   square root (s faithful, x > 0): the side of sqrt(x) is the sign of
//     x - s^2; sqrt(x) is past the midpoint m between s and its neighbour s'
//     exactly when x - s s' > 0 (upwards) or x - s' s <= 0 (downwards),
//     because x - m^2 = x - s s' - (s' - s)^2 / 4 and x - s s' is a multiple
//     of (s' - s)^2.
// On the host (where / and sqrt are IEEE) the same finishing steps are used
// by the CPU tests to check them on faithful-but-wrong inputs.
#pragma once
#pragma clang fp contract(off)

#include <cstring>

#include "wt_common.hpp"

namespace wt {

WT_HD long long bits_of(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __double_as_longlong(x);
#else
    long long b;
    std::memcpy(&b, &x, sizeof b);
    return b;
#endif
}

WT_HD double double_of(long long b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __longlong_as_double(b);
#else
    double x;
    std::memcpy(&x, &b, sizeof x);
    return x;
#endif
}

// Adjacent double of a finite non-zero x, towards +inf (up) or -inf.
WT_HD double neighbour(double x, bool up)
{
    const bool away = (x > 0.0) == up;          // magnitude grows
    return double_of(bits_of(x) + (away ? 1 : -1));
}

// Nearest double to a / b given a faithful q (b > 0).  An infinite or NaN q
// (overflow, or NaN operands) is already the IEEE result.
WT_HD double div_finish(double q, double a, double b)
{
    const double r = __builtin_fma(-q, b, a);
    if (!(r != 0.0) || !(q != 0.0) || !__builtin_isfinite(q)) return q;   // exact, 0, inf, NaN
    const double qn = neighbour(q, r > 0.0);
    const double rn = __builtin_fma(-qn, b, a);
    return __builtin_fabs(rn) < __builtin_fabs(r) ? qn : q;
}

// Nearest double to sqrt(x) given a faithful s (x > 0).
WT_HD double sqrt_finish(double s, double x)
{
    if (!(s > 0.0)) return s;
    const double r = __builtin_fma(-s, s, x);
    if (r > 0.0) {
        const double su = neighbour(s, true);
        return __builtin_fma(-s, su, x) > 0.0 ? su : s;
    }
    if (r < 0.0) {
        const double sd = neighbour(s, false);
        return __builtin_fma(-sd, s, x) <= 0.0 ? sd : s;
    }
    return s;
}

// a / b rounded to nearest from y = RN(1 / b) (b > 0): two FMA corrections
// (Markstein): q1 = q0 + (a - b q0) y is within one ulp of a / b, and with y
// the nearest reciprocal, q1 + (a - b q1) y rounds to the nearest quotient.
// Used where several quotients share a denominator.  Same code on the host,
// where the CPU tests check it against IEEE division.
WT_HD double div_by_recip(double a, double b, double y)
{
    const double q0 = a * y;
    const double q1 = __builtin_fma(__builtin_fma(-b, q0, a), y, q0);
    return __builtin_fma(__builtin_fma(-b, q1, a), y, q1);
}

// a / b rounded to nearest (b > 0 wherever the kernels divide).
WT_HD double div_rn(double a, double b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return div_finish(a / b, a, b);
#else
    return a / b;
#endif
}

// a / b rounded to nearest for a >= 0 and b > 0 from y = RN(1 / b), with the
// range of div_by_recip's proof checked: a = 0, or a and the first product
// both at least 2^-900 (the remainders a - b q are then exact) and the product
// far from overflow; otherwise (tiny, huge or NaN) the full division is taken.
WT_HD double div_by_recip_checked(double a, double b, double y)
{
    const double q0 = a * y;
    if ((a >= 0x1p-900 && q0 >= 0x1p-900 && q0 <= 0x1p+1000) || a == 0.0) {
        const double q1 = __builtin_fma(__builtin_fma(-b, q0, a), y, q0);
        return __builtin_fma(__builtin_fma(-b, q1, a), y, q1);
    }
    return div_rn(a, b);
}

// 1 / b rounded to nearest from an estimate y0 within 2^-14 (relative) of
// 1 / b, for 2^-1000 <= b <= 2^1000: two Newton steps (each squares the
// relative error, and their rounding errors stay far below an ulp) give a
// faithful reciprocal, and the exact neighbour test makes it the nearest.
WT_HD double recip_refine(double b, double y0)
{
    double y = __builtin_fma(y0, __builtin_fma(-b, y0, 1.0), y0);
    y = __builtin_fma(y, __builtin_fma(-b, y, 1.0), y);
    return div_finish(y, 1.0, b);
}

// 1 / b rounded to nearest for 2^-1000 <= b <= 2^1000: the hardware
// reciprocal estimate, refined.
WT_HD double recip_rn(double b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return recip_refine(b, __builtin_amdgcn_rcp(b));
#else
    return 1.0 / b;
#endif
}

// 1 / b for normal b (fast FP64 mode): the hardware estimate and two Newton steps,
// within an ulp or so of the nearest reciprocal, no exact finishing.
WT_HD double rcp_fast(double b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double y = __builtin_amdgcn_rcp(b);
    y = __builtin_fma(y, __builtin_fma(-b, y, 1.0), y);
    return __builtin_fma(y, __builtin_fma(-b, y, 1.0), y);
#else
    return 1.0 / b;
#endif
}

// 1/sqrt(x) for the fast forms (normal positive x): the hardware estimate and two
// Newton steps r <- r + (r / 2)(1 - (x r) r), the residual by a fused multiply-add.
// One of these gives a square root (x r), its reciprocal (r) and 1/x (r^2) together,
// where the compiler's square root takes range scaling, an iteration and a class
// fix-up, and a reciprocal its own estimate and steps.  Zero, infinite and negative x
// (states the kernels report as non-physical) give non-finite results.
WT_HD double rsq_fast(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rsq(x);
    double t = x * r;
    r = __builtin_fma(0.5 * r, __builtin_fma(-t, r, 1.0), r);
    t = x * r;
    return __builtin_fma(0.5 * r, __builtin_fma(-t, r, 1.0), r);
#else
    return 1.0 / __builtin_sqrt(x);
#endif
}

// Square root for the fast forms: x / sqrt(x) by the refined reciprocal square root
// (no exact finishing step; the rsq of the same x elsewhere is the same value, so a
// square root and a reciprocal of one quantity share it).
WT_HD double sqrt_fast(double x)
{
    return x * rsq_fast(x);
}

WT_HD double sqrt_rn(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return sqrt_finish(__builtin_sqrt(x), x);
#else
    return __builtin_sqrt(x);
#endif
}

}  // namespace wt
