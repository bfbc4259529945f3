// fastmath.hpp -- double-precision sine/cosine and reciprocal square root for
// the quadrature kernels (host and device).
//
// sincos_cw: Cody-Waite argument reduction by pi/2 (pi/2 split into three
// parts, the first two with 30 significant bits so that n * P1 and n * P2
// are exact for |n| < 2^23) followed by the Taylor series of sin and cos on
// [-pi/4, pi/4] through the r^17 and r^16 terms (truncation error below
// 1e-18 there) and a quadrant selection.  Intended for |x| < 1e6; larger
// arguments use the library routine.
//
// rsqrt_nr (device): the hardware reciprocal-square-root estimate refined by
// two Newton steps y <- y (3 - x y^2) / 2.
#pragma once

#include <cmath>

#ifndef NFQ_HD
#if defined(__HIPCC__)
#define NFQ_HD __host__ __device__
#else
#define NFQ_HD
#endif
#endif

namespace nfq {

NFQ_HD inline void sincos_cw(double x, double *sp, double *cp)
{
    // pi/2 = P1 + P2 + P3 (P1, P2: 30 significant bits)
    const double P1 = 0x1.921fb54000000p+0;
    const double P2 = 0x1.10b4611800000p-30;
    const double P3 = 0x1.313198a2e0370p-61;
    const double TWO_OVER_PI = 0x1.45f306dc9c883p-1;
    if (!(__builtin_fabs(x) < 1e6)) {
#if defined(__HIP_DEVICE_COMPILE__)
        sincos(x, sp, cp);
#else
        *sp = std::sin(x);
        *cp = std::cos(x);
#endif
        return;
    }
    const double nf = __builtin_rint(x * TWO_OVER_PI);
    double r = __builtin_fma(-nf, P1, x);
    r = __builtin_fma(-nf, P2, r);
    r = __builtin_fma(-nf, P3, r);
    const int q = (int)((long long)nf & 3);
    const double r2 = r * r;
    // sin r = r (1 + r2 (-1/3! + r2 (1/5! + ... + r2 / 17!)))
    double ps = 2.8114572543455206e-15;
    ps = __builtin_fma(ps, r2, -7.647163731819816e-13);
    ps = __builtin_fma(ps, r2, 1.6059043836821613e-10);
    ps = __builtin_fma(ps, r2, -2.505210838544172e-08);
    ps = __builtin_fma(ps, r2, 2.7557319223985893e-06);
    ps = __builtin_fma(ps, r2, -0.0001984126984126984);
    ps = __builtin_fma(ps, r2, 0.008333333333333333);
    ps = __builtin_fma(ps, r2, -0.16666666666666666);
    const double s = __builtin_fma(r * r2, ps, r);
    // cos r = 1 + r2 (-1/2! + r2 (1/4! + ... + r2 / 16!))
    double pc = 4.779477332387385e-14;
    pc = __builtin_fma(pc, r2, -1.1470745597729725e-11);
    pc = __builtin_fma(pc, r2, 2.08767569878681e-09);
    pc = __builtin_fma(pc, r2, -2.755731922398589e-07);
    pc = __builtin_fma(pc, r2, 2.48015873015873e-05);
    pc = __builtin_fma(pc, r2, -0.001388888888888889);
    pc = __builtin_fma(pc, r2, 0.041666666666666664);
    pc = __builtin_fma(pc, r2, -0.5);
    const double c = __builtin_fma(r2, pc, 1.0);
    const bool swap = (q & 1) != 0;
    const double ss = swap ? c : s, cc = swap ? s : c;
    *sp = (q == 2 || q == 3) ? -ss : ss;
    *cp = (q == 1 || q == 2) ? -cc : cc;
}

#if defined(__HIPCC__)
__device__ __forceinline__ double rsqrt_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    y = y * __builtin_fma(-hx * y, y, 1.5);
    y = y * __builtin_fma(-hx * y, y, 1.5);
    return y;
}
#endif

}  // namespace nfq
