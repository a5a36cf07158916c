// hankel_dev.h -- device evaluation of H0^(1)(k r) and H1^(1)(k r) for one
// wavenumber k (Im k >= 0) and many distances r > 0 (fundamental solution,
// eq. (fundamental_sol), and its derivative).
//
// Two regimes, chosen per lane by |k r| against XS:
//  * |k r| < XS: ascending series (DLMF 10.2.2, 10.8.1, 10.8.2) written as
//    polynomials in s = r^2 whose coefficients already carry the powers of k
//    (built once per wavenumber by the setup kernel):
//        J0 = sum j0_m s^m,        Y0 = (2/pi) ln r J0 + lk0 J0 + sum e0_m s^m,
//        J1 = r sum j1_m s^m,      Y1 = y1 / r + ((2/pi) ln r + lk1) J1 + r sum e1_m s^m;
//    ln(k r / 2) = ln r + ln(k / 2) splits the logarithm into a real part per
//    lane and a per-wavenumber constant.
//  * |k r| >= XS: H_nu = sqrt(2/(pi k)) r^{-1/2} e^{i(k r - nu pi/2 - pi/4)} P_nu,
//    P_nu = m_nu(w) + i (XS/(k r)) n_nu(w), w = (XS/(k r))^2, with m, n the
//    fitted amplitude polynomials; with rho = 1/r^2 they are polynomials in
//    rho whose (complex) coefficients are a_m (XS/k)^(2m).
// For real k every polynomial has real coefficients (CPLX = false); for lossy
// media the same code runs on complex coefficients (CPLX = true).
#pragma once

#include "internal.h"

namespace bemk {

struct cd {
    double re, im;
};

__device__ __forceinline__ cd cmul(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cd cadd(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cd cscale(cd a, double s) { return {a.re * s, a.im * s}; }

template <int N>
__device__ __forceinline__ double horner(const double* __restrict__ c, double x)
{
    double acc = c[N - 1];
#pragma unroll
    for (int m = N - 2; m >= 0; --m) acc = fma(acc, x, c[m]);
    return acc;
}

// complex coefficients (re[], im[]) at a real argument
template <int N>
__device__ __forceinline__ cd horner_c(const double* __restrict__ cr, const double* __restrict__ ci, double x)
{
    double ar = cr[N - 1], ai = ci[N - 1];
#pragma unroll
    for (int m = N - 2; m >= 0; --m) {
        ar = fma(ar, x, cr[m]);
        ai = fma(ai, x, ci[m]);
    }
    return {ar, ai};
}

// H0(k r), H1(k r).  r2 = r^2, rinv = 1/r, srinv = r^{-1/2}.
template <bool CPLX>
__device__ __forceinline__ void hankel01(const WaveConst& W, double r, double r2, double rinv, double srinv, cd& h0,
                                         cd& h1)
{
    constexpr double TWO_OVER_PI = 0.63661977236758134308;
    if (r2 < W.r2_small) {
        const double lnr = log(r);
        const double tl = TWO_OVER_PI * lnr;
        if (!CPLX) {
            const double j0 = horner<NSER>(W.j0r, r2);
            const double e0 = horner<NSER>(W.e0r, r2);
            const double j1 = r * horner<NSER>(W.j1r, r2);
            const double e1 = horner<NSER>(W.e1r, r2);
            const double y0 = fma(tl + W.lk0r, j0, e0);
            const double y1 = fma(W.y1r, rinv, fma(tl + W.lk1r, j1, r * e1));
            h0 = {j0, y0};
            h1 = {j1, y1};
        } else {
            const cd j0 = horner_c<NSER>(W.j0r, W.j0i, r2);
            const cd e0 = horner_c<NSER>(W.e0r, W.e0i, r2);
            cd j1 = horner_c<NSER>(W.j1r, W.j1i, r2);
            j1 = cscale(j1, r);
            const cd e1 = horner_c<NSER>(W.e1r, W.e1i, r2);
            const cd y0 = cadd(cmul({tl + W.lk0r, W.lk0i}, j0), e0);
            const cd y1 = cadd(cadd(cscale({W.y1r, W.y1i}, rinv), cmul({tl + W.lk1r, W.lk1i}, j1)), cscale(e1, r));
            h0 = {j0.re - y0.im, j0.im + y0.re};
            h1 = {j1.re - y1.im, j1.im + y1.re};
        }
    } else {
        const double rho = rinv * rinv;
        double sn, cs;
        sincos(W.kr * r, &sn, &cs);
        if (!CPLX) {
            const double m0 = horner<NAMP>(W.m0r, rho);
            const double n0 = horner<NAMP>(W.n0r, rho);
            const double m1 = horner<NAMP>(W.m1r, rho);
            const double n1 = horner<NAMP>(W.n1r, rho);
            const double u = W.ur * rinv;
            const cd e = {cs * srinv, sn * srinv};
            const cd p0 = {m0, u * n0};
            const cd p1 = {m1, u * n1};
            h0 = cmul(cmul(e, {W.a0r, W.a0i}), p0);
            h1 = cmul(cmul(e, {W.a1r, W.a1i}), p1);
        } else {
            const cd m0 = horner_c<NAMP>(W.m0r, W.m0i, rho);
            const cd n0 = horner_c<NAMP>(W.n0r, W.n0i, rho);
            const cd m1 = horner_c<NAMP>(W.m1r, W.m1i, rho);
            const cd n1 = horner_c<NAMP>(W.n1r, W.n1i, rho);
            const cd u = {W.ur * rinv, W.ui * rinv};
            const cd un0 = cmul(u, n0), un1 = cmul(u, n1);
            const cd p0 = {m0.re - un0.im, m0.im + un0.re};
            const cd p1 = {m1.re - un1.im, m1.im + un1.re};
            const double damp = exp(-W.ki * r) * srinv;
            const cd e = {cs * damp, sn * damp};
            h0 = cmul(cmul(e, {W.a0r, W.a0i}), p0);
            h1 = cmul(cmul(e, {W.a1r, W.a1i}), p1);
        }
    }
}

// H1 only (end-point terms of the hypersingular operator).
template <bool CPLX>
__device__ __forceinline__ cd hankel1_only(const WaveConst& W, double r, double r2, double rinv, double srinv)
{
    cd h0, h1;
    hankel01<CPLX>(W, r, r2, rinv, srinv, h0, h1);
    return h1;
}

}  // namespace bemk
