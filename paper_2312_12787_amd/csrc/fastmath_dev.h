// fastmath_dev.h -- FP64 square roots and sine/cosine for the assembly's
// large-argument path (distances between distinct boundary points, phases
// k r of moderate size).  Built from the hardware reciprocal-square-root
// estimate and fused multiply-adds only: no IEEE special-case fix-ups, no
// table lookups, every constant a compile-time literal.
//
// Domains: sqrt_rsqrt / rsqrt_nr take normal x > 0; sincos_cw takes
// |x| < 2^30 (the reduction below is exact there; the rounding of x itself,
// one ulp of k r, is the dominant error of any phase evaluation).
#pragma once

#include <hip/hip_runtime.h>

namespace bemk {

// r = sqrt(x) and ri = 1/sqrt(x): the v_rsq_f64 estimate y0 refined by two
// steps of Goldschmidt's coupled iteration, g -> sqrt(x), h -> 1/(2 sqrt(x)):
//   e = 1/2 - g h,  g <- g + g e,  h <- h + h e
// (quadratic convergence: a relative error eps of y0 leaves about eps^4).
__device__ __forceinline__ void sqrt_rsqrt(double x, double& r, double& ri)
{
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    double e = fma(-g, h, 0.5);
    g = fma(g, e, g);
    h = fma(h, e, h);
    e = fma(-g, h, 0.5);
    g = fma(g, e, g);
    h = fma(h, e, h);
    r = g;
    ri = h + h;
}

// 1/sqrt(x): the v_rsq_f64 estimate refined by two Newton steps for
// f(y) = 1/y^2 - x,  y <- y + (y/2)(1 - x y^2).
__device__ __forceinline__ double rsqrt_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double e = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    return y;
}

// sin x and cos x.  Cody and Waite's additive reduction x = n pi/2 + t with
// pi/2 split into P1 = pi/2 rounded to double and P2 = pi/2 - P1 rounded:
// with a fused multiply-add, x - n P1 is exact (both are integer multiples of
// 2^-52 below 2 in magnitude once |x| >= 1, and n = 0 below), and n P2 leaves
// an error of about n 1.5e-33.  On |t| <= pi/4 (+ rounding) the Taylor series
//   sin t = t - t^3/3! + ... - t^15/15! + t^17/17!   (truncation < 1e-19)
//   cos t = 1 - t^2/2! + ... + t^16/16!              (truncation < 3e-18)
// in u = t^2, then the quadrant n mod 4 swaps and negates.
__device__ __forceinline__ void sincos_cw(double x, double& s, double& c)
{
    constexpr double TWO_OVER_PI = 0x1.45f306dc9c883p-1;  // 2/pi
    constexpr double P1 = 0x1.921fb54442d18p+0;           // pi/2 rounded to double
    constexpr double P2 = 0x1.1a62633145c07p-54;          // pi/2 - P1 rounded to double
    const double n = rint(x * TWO_OVER_PI);
    double t = fma(-n, P1, x);
    t = fma(-n, P2, t);
    const double u = t * t;
    // (-1)^m / (2m+1)!, m = 1..8, and (-1)^m / (2m)!, m = 1..8 (factorials exact in double)
    double ps = 1.0 / 355687428096000.0;   // 1/17!
    ps = fma(ps, u, -1.0 / 1307674368000.0);  // 1/15!
    ps = fma(ps, u, 1.0 / 6227020800.0);      // 1/13!
    ps = fma(ps, u, -1.0 / 39916800.0);       // 1/11!
    ps = fma(ps, u, 1.0 / 362880.0);          // 1/9!
    ps = fma(ps, u, -1.0 / 5040.0);           // 1/7!
    ps = fma(ps, u, 1.0 / 120.0);             // 1/5!
    ps = fma(ps, u, -1.0 / 6.0);              // 1/3!
    double pc = 1.0 / 20922789888000.0;    // 1/16!
    pc = fma(pc, u, -1.0 / 87178291200.0);    // 1/14!
    pc = fma(pc, u, 1.0 / 479001600.0);       // 1/12!
    pc = fma(pc, u, -1.0 / 3628800.0);        // 1/10!
    pc = fma(pc, u, 1.0 / 40320.0);           // 1/8!
    pc = fma(pc, u, -1.0 / 720.0);            // 1/6!
    pc = fma(pc, u, 1.0 / 24.0);              // 1/4!
    pc = fma(pc, u, -0.5);                    // 1/2!
    const double st = fma(t * u, ps, t);
    const double ct = fma(u, pc, 1.0);
    // x = n pi/2 + t:  q = n mod 4;  sin x = (q odd ? cos t : sin t) (-1)^[q in {2,3}],
    //                                cos x = (q odd ? sin t : cos t) (-1)^[q in {1,2}]
    // (two's complement: the low bits of a negative n are n mod 4 as well)
    const unsigned q = (unsigned)(int)n;
    const double a = (q & 1u) ? ct : st;
    const double b = (q & 1u) ? st : ct;
    s = __hiloint2double((int)((unsigned)__double2hiint(a) ^ ((q & 2u) << 30)), __double2loint(a));
    c = __hiloint2double((int)((unsigned)__double2hiint(b) ^ (((q + 1u) & 2u) << 30)), __double2loint(b));
}

}  // namespace bemk
