// hankel_dev.h -- device evaluation of H0^(1)(k r) and H1^(1)(k r) for one
// wavenumber k (Im k >= 0) and many distances r > 0 (fundamental solution,
// eq. (fundamental_sol), and its derivative).
//
// Every polynomial has compile-time real coefficients (hankel_tables.h); the
// wavenumber enters only through the argument, so a launch keeps a handful
// of per-wavenumber constants (WaveConst) instead of coefficient tables.
//  * |k r| < XS: ascending series (DLMF 10.2.2, 10.8.1, 10.8.2) in
//    t = (k r / 2)^2 = (k/2)^2 r^2:
//        J0 = J0(t),  Y0 = (2/pi)(ln(kr/2) + gamma) J0 + E0(t),
//        J1 = (kr/2) J1(t),  Y1 = -(2/pi)/(k r) + (2/pi) ln(kr/2) J1 + (kr/2) E1(t),
//    with ln(kr/2) = ln r + ln(k/2) (a real logarithm per lane);
//  * |k r| >= XS: H_nu = sqrt(2/(pi k)) r^{-1/2} e^{i(k r - nu pi/2 - pi/4)} P_nu,
//    P_nu = m_nu(w) + i (XS/(k r)) n_nu(w),  w = (XS/k)^2 / r^2, with m, n the
//    fitted amplitude polynomials.
// Real k: Horner in a real argument.  Complex k (lossy media): the same real
// polynomials at a complex argument z = x + i y by dividing out the quadratic
// z^2 - 2 x z + |z|^2 (Knuth's scheme): two multiply-adds per coefficient.
#pragma once

#include "fastmath_dev.h"
#include "hankel_tables.h"
#include "internal.h"

namespace bemk {

struct cd {
    double re, im;
};

__device__ __forceinline__ cd cmul(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cd cadd(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cd cscale(cd a, double s) { return {a.re * s, a.im * s}; }

// sum_m c[m] x^m, x real (c: an array of N coefficients, in any address space)
template <int N, class C, class T>
__device__ __forceinline__ T poly_n(const C& c, T x)
{
    T acc = c[N - 1];
#pragma unroll
    for (int m = N - 2; m >= 0; --m) acc = fma(acc, x, (T)c[m]);
    return acc;
}
template <int N, class T>
__device__ __forceinline__ T poly_real(const T (&c)[N], T x)
{
    return poly_n<N>(c, x);
}

// sum_m c[m] z^m at complex z = x + i y for real c: with R = 2x, S = |z|^2,
// b_{N-1} = c_{N-1}, b_{N-2} = c_{N-2} + R b_{N-1}, b_m = c_m + R b_{m+1} - S b_{m+2},
// p(z) = (x b_1 + c_0 - S b_2) + i y b_1.   (N >= 3)
template <int N, class C, class T>
__device__ __forceinline__ void poly_cplx_n(const C& c, T x, T y, T R, T S, T& pr, T& pi)
{
    T b2 = c[N - 1];
    T b1 = fma(R, b2, (T)c[N - 2]);
#pragma unroll
    for (int m = N - 3; m >= 1; --m) {
        const T b0 = fma(R, b1, fma(-S, b2, (T)c[m]));
        b2 = b1;
        b1 = b0;
    }
    pr = fma(x, b1, fma(-S, b2, (T)c[0]));
    pi = y * b1;
}
template <int N, class T>
__device__ __forceinline__ void poly_cplx(const T (&c)[N], T x, T y, T R, T S, T& pr, T& pi)
{
    poly_cplx_n<N>(c, x, y, R, S, pr, pi);
}

// The ascending-series coefficients as one object in device memory.  The
// general evaluator can read them through a pointer the compiler must reload
// on each call (scalar loads, nothing held in registers across a loop), for
// paths that run rarely and would otherwise keep 88 coefficients resident.
struct HankelTabs {
    double j0[SERIES_NC], e0[SERIES_NC], j1[SERIES_NC], e1[SERIES_NC];
};
constexpr HankelTabs make_hankel_tabs()
{
    HankelTabs t{};
    for (int m = 0; m < SERIES_NC; ++m) {
        t.j0[m] = SERIES_J0[m];
        t.e0[m] = SERIES_E0[m];
        t.j1[m] = SERIES_J1[m];
        t.e1[m] = SERIES_E1[m];
    }
    return t;
}
static __device__ const HankelTabs g_hankel_tabs = make_hankel_tabs();
typedef const __attribute__((address_space(4))) HankelTabs* HankelTabsPtr;
__device__ __forceinline__ HankelTabsPtr hankel_tabs_fresh()
{
    HankelTabsPtr t = (HankelTabsPtr)&g_hankel_tabs;
    asm volatile("" : "+s"(t));  // opaque: loads through t are not hoisted out of loops
    return t;
}

// sum_m c[m] w^m from shared powers p[m] = w^m (p[0] unused), highest degree
// first.  The accumulator is the only register each step overwrites (Horner's
// rule overwrites a copy of the constant instead).  Used where 0 < w <= 1 and
// the |c[m]| of m >= 1 are small, so the order costs no accuracy.
template <int N, class T>
__device__ __forceinline__ T poly_pow(const T (&c)[N], const T (&p)[N])
{
    T acc = c[N - 1] * p[N - 1];
#pragma unroll
    for (int m = N - 2; m >= 1; --m) acc = fma(c[m], p[m], acc);
    return acc + c[0];
}

// Large-argument form for |k r| >= XS, from r, 1/r and r^{-1/2}.  The phase
// phi = Re(k) r - pi/4 is reduced once for both orders:
//   H0 = A r^{-1/2} e^{i phi} (m0 + i u n0),
//   H1 = A r^{-1/2} e^{i phi} (-i) (m1 + i u n1),   u = XS/(k r),
// A = sqrt(2/(pi k)), times e^{-Im(k) r} for complex k.  H0 is skipped when
// only H1 is wanted.
template <bool CPLX, bool WANT_H0>
__device__ __forceinline__ void hankel_asym(const WaveConst& W, double r, double rinv, double sr, cd& h0, cd& h1)
{
    constexpr double PI_4 = 0x1.921fb54442d18p-1;
    double sn, cs;
    sincos_cw(fma(W.kr, r, -PI_4), sn, cs);
    const double rho = rinv * rinv;
    if (!CPLX) {
        // w = (XS/(k r))^2 <= 1; its powers are shared by the four amplitude polynomials
        double p[HANKEL_NC_F64];
        p[1] = W.wr * rho;
#pragma unroll
        for (int m = 2; m < HANKEL_NC_F64; ++m) p[m] = p[m / 2] * p[m - m / 2];
        const double u = W.ur * rinv;
        const double a = W.ampr * sr;
        const double er = cs * a, ei = sn * a;
        const double m1 = poly_pow(HANKEL_M1_F64, p), un1 = u * poly_pow(HANKEL_N1_F64, p);
        h1 = {fma(er, un1, ei * m1), fma(ei, un1, -er * m1)};
        if (WANT_H0) {
            const double m0 = poly_pow(HANKEL_M0_F64, p), un0 = u * poly_pow(HANKEL_N0_F64, p);
            h0 = {fma(er, m0, -ei * un0), fma(er, un0, ei * m0)};
        }
    } else {
        const double x = W.wr * rho, y = W.wi * rho;
        const double R = 2.0 * x, S = fma(x, x, y * y);
        const cd u = {W.ur * rinv, W.ui * rinv};
        const double damp = exp(-W.ki * r) * sr;
        const cd e = cmul({cs * damp, sn * damp}, {W.ampr, W.ampi});
        cd m1, n1;
        poly_cplx(HANKEL_M1_F64, x, y, R, S, m1.re, m1.im);
        poly_cplx(HANKEL_N1_F64, x, y, R, S, n1.re, n1.im);
        const cd un1 = cmul(u, n1);
        h1 = cmul(e, {m1.im + un1.re, un1.im - m1.re});
        if (WANT_H0) {
            cd m0, n0;
            poly_cplx(HANKEL_M0_F64, x, y, R, S, m0.re, m0.im);
            poly_cplx(HANKEL_N0_F64, x, y, R, S, n0.re, n0.im);
            const cd un0 = cmul(u, n0);
            h0 = cmul(e, {m0.re - un0.im, m0.im + un0.re});
        }
    }
}

// H0(k r) and H1(k r) when |k r| >= XS is known for the pair (no per-lane
// branch, no series), from the offset (rx, ry) = x - y; returns 1/r.
template <bool CPLX, bool WANT_H0>
__device__ __forceinline__ double hankel01_far(const WaveConst& W, double rx, double ry, cd& h0, cd& h1)
{
    const double r2 = fma(rx, rx, ry * ry);
    double r, rinv;
    sqrt_rsqrt(r2, r, rinv);
    hankel_asym<CPLX, WANT_H0>(W, r, rinv, rsqrt_nr(r), h0, h1);
    return rinv;
}

// H0(k r), H1(k r).  r2 = r^2, rinv = 1/r, srinv = r^{-1/2}.  Below XS the
// ascending series (MEM: its coefficients from g_hankel_tabs by scalar loads
// instead of immediates), above it hankel_asym.
template <bool CPLX, bool MEM = false>
__device__ __forceinline__ void hankel01(const WaveConst& W, double r, double r2, double rinv, double srinv, cd& h0,
                                         cd& h1)
{
    HankelTabsPtr T = nullptr;
    if (MEM) T = hankel_tabs_fresh();
    constexpr double TWO_OVER_PI = 0.63661977236758134308;
    constexpr double EULER = 0.57721566490153286061;
    // both branches set these scalars and h0, h1 are written once after the
    // join: stores to different fields at the ends of the two branches would
    // be merged into one store through a selected address, which keeps the
    // caller's h0, h1 in scratch memory
    double h0r, h0i, h1r, h1i;
    if (r2 < W.r2_small) {
        const double lnr = log(r);
        if (!CPLX) {
            const double t = W.tr * r2;
            const double j0 = MEM ? poly_n<SERIES_NC>(T->j0, t) : poly_real(SERIES_J0, t);
            const double e0 = MEM ? poly_n<SERIES_NC>(T->e0, t) : poly_real(SERIES_E0, t);
            const double zh = W.hr * r;
            const double j1 = zh * (MEM ? poly_n<SERIES_NC>(T->j1, t) : poly_real(SERIES_J1, t));
            const double e1 = MEM ? poly_n<SERIES_NC>(T->e1, t) : poly_real(SERIES_E1, t);
            const double lz = lnr + W.lkr;
            const double y0 = fma(TWO_OVER_PI * (lz + EULER), j0, e0);
            const double y1 = fma(W.y1r, rinv, fma(TWO_OVER_PI * lz, j1, zh * e1));
            h0r = j0;
            h0i = y0;
            h1r = j1;
            h1i = y1;
        } else {
            const double x = W.tr * r2, y = W.ti * r2;
            const double R = 2.0 * x, S = fma(x, x, y * y);
            cd j0, e0, p1, e1;
            if (MEM)
                poly_cplx_n<SERIES_NC>(T->j0, x, y, R, S, j0.re, j0.im);
            else
                poly_cplx(SERIES_J0, x, y, R, S, j0.re, j0.im);
            if (MEM)
                poly_cplx_n<SERIES_NC>(T->e0, x, y, R, S, e0.re, e0.im);
            else
                poly_cplx(SERIES_E0, x, y, R, S, e0.re, e0.im);
            if (MEM)
                poly_cplx_n<SERIES_NC>(T->j1, x, y, R, S, p1.re, p1.im);
            else
                poly_cplx(SERIES_J1, x, y, R, S, p1.re, p1.im);
            if (MEM)
                poly_cplx_n<SERIES_NC>(T->e1, x, y, R, S, e1.re, e1.im);
            else
                poly_cplx(SERIES_E1, x, y, R, S, e1.re, e1.im);
            const cd zh = {W.hr * r, W.hi * r};
            const cd j1 = cmul(zh, p1);
            const cd lz = {lnr + W.lkr, W.lki};
            const cd y0 = cadd(cmul({TWO_OVER_PI * (lz.re + EULER), TWO_OVER_PI * lz.im}, j0), e0);
            const cd y1 = cadd(cadd(cscale({W.y1r, W.y1i}, rinv), cmul(cscale(lz, TWO_OVER_PI), j1)), cmul(zh, e1));
            h0r = j0.re - y0.im;
            h0i = j0.im + y0.re;
            h1r = j1.re - y1.im;
            h1i = j1.im + y1.re;
        }
    } else {
        cd a0, a1;
        hankel_asym<CPLX, true>(W, r, rinv, srinv, a0, a1);
        h0r = a0.re;
        h0i = a0.im;
        h1r = a1.re;
        h1i = a1.im;
    }
    h0 = {h0r, h0i};
    h1 = {h1r, h1i};
}

// H1 only (end-point terms of the hypersingular operator).
template <bool CPLX, bool MEM = false>
__device__ __forceinline__ cd hankel1_only(const WaveConst& W, double r, double r2, double rinv, double srinv)
{
    cd h0, h1;
    hankel01<CPLX, MEM>(W, r, r2, rinv, srinv, h0, h1);
    return h1;
}

}  // namespace bemk
