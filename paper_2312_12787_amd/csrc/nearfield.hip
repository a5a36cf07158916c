// nearfield.hip -- the field at points off the boundary (Sec. 7.1: the total
// field at field points), from the boundary data of a solution.
//
// A point x of domain d takes the representation formula of that domain:
//   u(x) = [d = host] u_in(x) + sum_m sigma_dm sum_{j in m} (eps_d S_j(x) w_j - D_j(x) u_j),
//   S_j(x) = int_j G_d(x - y) ds_y,  D_j(x) = int_j dG_d/dn_y(x - y) ds_y,
// sigma_dm = +1 where the normal of interface m leaves domain d.
// Element integrals: the element's q-point Gauss rule when x is at least two
// element lengths away (Bernstein-ellipse error below 1e-14); closer, the
// Laplace parts of the kernels, -(1/2pi) ln r and (1/2pi) (x-y).n / r^2, and
// the next log terms, (k^2/8pi) r^2 ln r of the single layer and
// -(k^2/4pi) (x-y).n ln r of the double layer, are integrated in closed form
// over the straight element and Gauss is applied to what remains of
// (i/4) H0(kr) and (ik/4) H1(kr) (x-y).n / r, on each side of the foot of the
// perpendicular from x.
//
// Layout: points xy[2 p], xy[2 p + 1], domain dom[p]; X column-major [u; w]
// per right-hand side (ldx); U column-major, point fastest (ldu).  One wave
// per point: its 64 lanes take every 64th source element of each interface
// and a fixed-order butterfly adds their sums (a 101 x 101 grid is ~2550
// workgroups of four points, enough to fill the chip).  One launch per domain
// (uniform wavenumber and Hankel constants); points of other domains return
// at once, wave-uniformly.
#include <hip/hip_runtime.h>

#include "hankel_dev.h"
#include "internal.h"
#include "launch.h"

namespace bemk {

namespace {

constexpr int NF_BS = 256;
constexpr double INV_2PI = 0.15915494309189533577;

template <class T>
__device__ __forceinline__ const T* tab(const char* g, size_t off) { return reinterpret_cast<const T*>(g + off); }

// int_{u0}^{u1} ln sqrt(u^2 + xn^2) du
__device__ __forceinline__ double log_integral(double u0, double u1, double xn)
{
    auto F = [&](double u) {
        const double r2 = fma(u, u, xn * xn);
        double v = (u != 0.0 ? u * 0.5 * log(r2) : 0.0) - u;
        if (xn != 0.0) v += xn * atan(u / xn);
        return v;
    };
    return F(u1) - F(u0);
}

// int_{u0}^{u1} (u^2 + xn^2) ln sqrt(u^2 + xn^2) du
__device__ __forceinline__ double r2log_integral(double u0, double u1, double xn)
{
    const double d2 = xn * xn;
    auto F = [&](double u) {
        const double r2 = fma(u, u, d2);
        const double u3 = u * u * u;
        double v = (u != 0.0 ? (u3 / 6.0 + d2 * u * 0.5) * log(r2) : 0.0) - u3 / 9.0 + d2 * u / 3.0 - d2 * u;
        if (xn != 0.0) v += (d2 * xn - d2 * xn / 3.0) * atan(u / xn);
        return v;
    };
    return F(u1) - F(u0);
}

// The Gauss points of the element are formed here from its midpoint, tangent
// and length and the shared rule (as the geometry tables form them): lanes
// take different elements, and reading per-element point tables would cost
// one scattered load per point and coordinate.
template <bool CPLX>
__device__ __forceinline__ void element_integrals(const WaveConst& W, cd k, const ElemRec& E,
                                                  const double* __restrict__ gl, int q, double x, double y, cd& S,
                                                  cd& D)
{
    const double dx = x - E.ax, dy = y - E.ay;
    const double xt = dx * E.tx + dy * E.ty;  // along the element from node a
    const double xn = dx * E.nx + dy * E.ny;  // (x - y).n for every y on the element
    const double h = E.h;
    const double ut = xt < 0.0 ? -xt : (xt > h ? xt - h : 0.0);
    const double dist = sqrt(fma(ut, ut, xn * xn));
    const cd ik4 = {-0.25 * k.im, 0.25 * k.re};
    S = {0.0, 0.0};
    D = {0.0, 0.0};
    if (dist >= 2.0 * h) {
        const double cx = E.cx, cy = E.cy, tx = E.tx, ty = E.ty, hh = 0.5 * h;
        for (int g = 0; g < q; ++g) {
            const double sg = hh * gl[g];
            const double rx = x - (cx + sg * tx), ry = y - (cy + sg * ty);
            const double r2 = fma(rx, rx, ry * ry);
            double r, rinv;
            sqrt_rsqrt(r2, r, rinv);
            cd h0, h1;
            hankel01<CPLX, true>(W, r, r2, rinv, rsqrt_nr(r), h0, h1);
            const double wg = hh * gl[QMAX + g];
            S.re = fma(wg, h0.re, S.re);
            S.im = fma(wg, h0.im, S.im);
            const double wd = wg * (rx * E.nx + ry * E.ny) * rinv;
            D.re = fma(wd, h1.re, D.re);
            D.im = fma(wd, h1.im, D.im);
        }
        // S = (i/4) sum w H0, D = (ik/4) sum w H1 (r.n)
        S = {-0.25 * S.im, 0.25 * S.re};
        D = cmul(ik4, D);
        return;
    }
    // Laplace parts in closed form, and the log term of the double layer:
    // (ik/4) H1(kr) xn / r = xn / (2 pi r^2) - (k^2 / 4 pi) xn ln r + smooth
    const double lnint = log_integral(-xt, h - xt, xn);
    const double SL = -INV_2PI * lnint;
    const double DL = INV_2PI * atan2(xn * h, fma(xn, xn, -xt * (h - xt)));
    const cd k2 = cmul(k, k);
    const cd c4 = cscale(k2, 0.5 * INV_2PI * xn);  // (k^2 / 4 pi) xn
    const cd DLog = cscale(c4, -lnint);
    // and of the single layer: (1/2pi) ln r (1 - J0(kr)) = (k^2 / 8 pi) r^2 ln r + O(r^4 ln r)
    const cd c8 = cscale(k2, 0.25 * INV_2PI);       // k^2 / 8 pi
    const cd SLog = cscale(c8, r2log_integral(-xt, h - xt, xn));
    // smooth remainders by Gauss on [0, s*] and [s*, h] (s* = foot of the perpendicular)
    const double cut = fmin(fmax(xt, 0.0), h);
    cd sr = {0.0, 0.0}, dr = {0.0, 0.0};
    for (int part = 0; part < 2; ++part) {
        const double s0 = part == 0 ? 0.0 : cut, s1 = part == 0 ? cut : h;
        const double half = 0.5 * (s1 - s0), mid = 0.5 * (s0 + s1);
        if (half <= 0.0) continue;
        for (int g = 0; g < q; ++g) {
            const double s = fma(half, gl[g], mid);
            const double u = xt - s;  // (x - y).t
            const double r2 = fma(u, u, xn * xn);
            double r, rinv;
            sqrt_rsqrt(r2, r, rinv);
            cd h0, h1;
            hankel01<CPLX, true>(W, r, r2, rinv, rsqrt_nr(r), h0, h1);
            const double wg = half * gl[QMAX + g];
            // (i/4) H0 + (1/2pi) ln r - (k^2 / 8 pi) r^2 ln r
            const double lnr = log(r);
            const double lr2 = wg * r2 * lnr;
            sr.re = fma(wg, -0.25 * h0.im + INV_2PI * lnr, fma(-lr2, c8.re, sr.re));
            sr.im = fma(wg, 0.25 * h0.re, fma(-lr2, c8.im, sr.im));
            // [(ik/4) H1 - 1/(2 pi r)] xn / r + (k^2 / 4 pi) xn ln r
            const cd a = cmul(ik4, h1);
            const double f = wg * xn * rinv;
            const double lr = wg * lnr;
            dr.re = fma(f, a.re - INV_2PI * rinv, fma(lr, c4.re, dr.re));
            dr.im = fma(f, a.im, fma(lr, c4.im, dr.im));
        }
    }
    S = {sr.re + SL + SLog.re, sr.im + SLog.im};
    D = {dr.re + DL + DLog.re, dr.im + DLog.im};
}

// sum over the wave's 64 lanes in a fixed butterfly order (every lane ends
// with the same value)
__device__ __forceinline__ double wave_add(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <bool CPLX>
__global__ __launch_bounds__(NF_BS, 2) void k_nearfield(const char* __restrict__ g, GeomLayout L, int n_if, int N, int q,
                                                   int d,
                                                   const double2* __restrict__ X, size_t ldx, int nr,
                                                   NearAngles ang, int add_incident, const double* __restrict__ xy,
                                                   const int* __restrict__ dom, int npts, double2* __restrict__ U,
                                                   size_t ldu)
{
    const int lane = threadIdx.x & 63;
    const int p = blockIdx.x * (NF_BS / 64) + (threadIdx.x >> 6);
    if (p >= npts || dom[p] != d) return;  // uniform over the wave
    const double x = xy[2 * (size_t)p], y = xy[2 * (size_t)p + 1];
    const WaveConst W = tab<WaveConst>(g, L.wave)[d];
    const DomConst Dm = tab<DomConst>(g, L.dom)[d];
    const cd k = {Dm.k[0], Dm.k[1]};
    const cd eps = {Dm.eps[0], Dm.eps[1]};
    const ElemRec* el = tab<ElemRec>(g, L.elem);
    const double* gl = tab<double>(g, L.gl);
    cd acc[NF_RB];
#pragma unroll
    for (int r = 0; r < NF_RB; ++r) acc[r] = {0.0, 0.0};
    for (int m = 0; m < n_if; ++m) {
        const int sg = tab<int>(g, L.sigma)[d * n_if + m];
        if (sg == 0) continue;
        const IfacePlan P = tab<IfacePlan>(g, L.iface)[m];
        for (int e = lane; e < P.count; e += 64) {
            const int j = P.off + e;
            cd S, D;
            element_integrals<CPLX>(W, k, el[j], gl, q, x, y, S, D);
            const cd eS = cscale(cmul(eps, S), (double)sg);
            const cd sD = cscale(D, (double)sg);
#pragma unroll
            for (int r = 0; r < NF_RB; ++r) {
                if (r < nr) {
                    const double2 u = X[(size_t)r * ldx + j], w = X[(size_t)r * ldx + N + j];
                    acc[r].re += eS.re * w.x - eS.im * w.y - (sD.re * u.x - sD.im * u.y);
                    acc[r].im += eS.re * w.y + eS.im * w.x - (sD.re * u.y + sD.im * u.x);
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < NF_RB; ++r) {
        if (r >= nr) continue;
        cd v = {wave_add(acc[r].re), wave_add(acc[r].im)};
        if (d == 0 && add_incident) {
            double sn, cs;
            sincos(ang.v[r], &sn, &cs);
            double ps, pc;
            sincos(k.re * (cs * x + sn * y), &ps, &pc);
            v.re += pc;
            v.im += ps;
        }
        if (lane == 0) U[(size_t)r * ldu + p] = make_double2(v.re, v.im);
    }
}

}  // namespace

hipError_t launch_nearfield(const char* g, const GeomLayout& L, int n_if, int n_dom, int N, int q, const int* dom_cplx,
                            const double2* X, size_t ldx, int nrhs, const double* angles, const double* xy,
                            const int* dom, int npts, double2* U, size_t ldu, hipStream_t s)
{
    const dim3 grid((npts + NF_BS / 64 - 1) / (NF_BS / 64));  // one wave per point
    for (int r0 = 0; r0 < nrhs; r0 += NF_RB) {
        const int nr = nrhs - r0 < NF_RB ? nrhs - r0 : NF_RB;
        NearAngles ang{};
        for (int r = 0; r < nr; ++r) ang.v[r] = angles ? angles[r0 + r] : 0.0;
        for (int d = 0; d < n_dom; ++d) {
            if (dom_cplx[d])
                hipLaunchKernelGGL(k_nearfield<true>, grid, dim3(NF_BS), 0, s, g, L, n_if, N, q, d, X + (size_t)r0 * ldx,
                                   ldx, nr, ang, angles ? 1 : 0, xy, dom, npts, U + (size_t)r0 * ldu, ldu);
            else
                hipLaunchKernelGGL(k_nearfield<false>, grid, dim3(NF_BS), 0, s, g, L, n_if, N, q, d,
                                   X + (size_t)r0 * ldx, ldx, nr, ang, angles ? 1 : 0, xy, dom, npts,
                                   U + (size_t)r0 * ldu, ldu);
        }
    }
    return hipGetLastError();
}

}  // namespace bemk
