// assemble.hip -- setup kernels (element table, Gauss rule, per-domain
// constants, self terms) and the fused assembly of the collocation matrix
// of the Calderon-ordered Burton-Miller system (Secs. 3-7 of arXiv 2312.12787).
#include <hip/hip_runtime.h>

#include "hankel_dev.h"
#include "hankel_tables.h"
#include "internal.h"
#include "launch.h"

namespace bemk {

namespace {

constexpr double PI = 3.14159265358979323846;
constexpr double EULER = 0.57721566490153286061;
// Assembly kernels: minimum waves per SIMD (1: the compiler may keep every
// polynomial coefficient and two interleaved Gauss points in registers; a
// higher floor forces scratch spills, measured 2-7x slower on gfx950) and
// Gauss points unrolled together.
#ifndef ASM_WAVES_PER_SIMD
#define ASM_WAVES_PER_SIMD 1
#endif
#ifndef ASM_GAUSS_UNROLL
#define ASM_GAUSS_UNROLL 2
#endif

template <class T>
__device__ __forceinline__ const T* tab(const char* g, size_t off) { return reinterpret_cast<const T*>(g + off); }
template <class T>
__device__ __forceinline__ T* tabw(char* g, size_t off) { return reinterpret_cast<T*>(g + off); }

__device__ __forceinline__ cd cdiv(cd a, cd b)
{
    const double den = b.re * b.re + b.im * b.im;
    return {(a.re * b.re + a.im * b.im) / den, (a.im * b.re - a.re * b.im) / den};
}
__device__ __forceinline__ cd csqrt_(cd z)
{
    const double r = hypot(z.re, z.im);
    double sr = sqrt(0.5 * (r + fabs(z.re)));
    if (sr == 0.0) return {0.0, 0.0};
    if (z.re >= 0.0) return {sr, z.im / (2.0 * sr)};
    return {fabs(z.im) / (2.0 * sr), z.im >= 0.0 ? sr : -sr};
}
__device__ __forceinline__ cd clog_(cd z) { return {log(hypot(z.re, z.im)), atan2(z.im, z.re)}; }

// ---------------------------------------------------------------------------
// Gauss-Legendre rule on [-1, 1] (Sec. 7).  One lane per node: Newton's
// method on P_q with P_q, P_q' from the three-term recurrence.
// ---------------------------------------------------------------------------
__global__ void k_gauss_rule(int q, double* gl)
{
    const int i = threadIdx.x;
    if (i >= q) return;
    double x = cos(PI * (4.0 * i + 3.0) / (4.0 * q + 2.0));
    double dp = 1.0;
    for (int it = 0; it < 60; ++it) {
        double p0 = 1.0, p1 = x;
        for (int n = 2; n <= q; ++n) {
            const double p2 = ((2.0 * n - 1.0) * x * p1 - (n - 1.0) * p0) / n;
            p0 = p1;
            p1 = p2;
        }
        const double pq = (q == 1) ? x : p1;
        const double pqm1 = (q == 1) ? 1.0 : p0;
        dp = q * (pqm1 - x * pq) / (1.0 - x * x);
        const double dx = pq / dp;
        x -= dx;
        if (fabs(dx) < 1e-17) break;
    }
    // recompute the derivative at the converged node
    double p0 = 1.0, p1 = x;
    for (int n = 2; n <= q; ++n) {
        const double p2 = ((2.0 * n - 1.0) * x * p1 - (n - 1.0) * p0) / n;
        p0 = p1;
        p1 = p2;
    }
    const double pq = (q == 1) ? x : p1, pqm1 = (q == 1) ? 1.0 : p0;
    dp = q * (pqm1 - x * pq) / (1.0 - x * x);
    // node i counted from the right end: store in ascending order
    gl[q - 1 - i] = x;
    gl[QMAX + q - 1 - i] = 2.0 / ((1.0 - x * x) * dp * dp);
}

// ---------------------------------------------------------------------------
// Element table and the Gauss points of every element (Secs. 4, 7).
// ---------------------------------------------------------------------------
__global__ void k_elements(char* g, GeomLayout L, int N, int q)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= N) return;
    const double2* nodes = tab<double2>(g, L.nodes);
    const int2 ab = tab<int2>(g, L.elnodes)[e];
    const double* gl = tab<double>(g, L.gl);
    const double2 a = nodes[ab.x], b = nodes[ab.y];
    ElemRec E;
    E.ax = a.x;
    E.ay = a.y;
    E.bx = b.x;
    E.by = b.y;
    E.cx = 0.5 * (a.x + b.x);
    E.cy = 0.5 * (a.y + b.y);
    const double dx = b.x - a.x, dy = b.y - a.y;
    E.h = sqrt(dx * dx + dy * dy);
    E.tx = dx / E.h;
    E.ty = dy / E.h;
    E.nx = -E.ty;
    E.ny = E.tx;
    for (int k = 0; k < 5; ++k) E.pad[k] = 0.0;
    tabw<ElemRec>(g, L.elem)[e] = E;
    GaussRec G;
    GaussRec32 G32;
    for (int k = 0; k < QMAX; ++k) {
        if (k < q) {
            const double s = 0.5 * E.h * gl[k];
            G.x[k] = E.cx + s * E.tx;
            G.y[k] = E.cy + s * E.ty;
            G.w[k] = 0.5 * E.h * gl[QMAX + k];
        } else {
            G.x[k] = G.y[k] = G.w[k] = 0.0;
        }
        G32.x[k] = (float)G.x[k];
        G32.y[k] = (float)G.y[k];
        G32.w[k] = (float)G.w[k];
    }
    tabw<GaussRec>(g, L.gauss)[e] = G;
    tabw<GaussRec32>(g, L.gauss32)[e] = G32;
}

// ---------------------------------------------------------------------------
// Per-domain constants: eps_d = (k_d/k_0)^2 (Sec. 2), the Burton-Miller
// coefficient alpha/eps_d (Sec. 6 recipe), the row scaling beta (Sec. 5) and
// the Hankel tables of the wavenumber.
// ---------------------------------------------------------------------------
__device__ void build_wave(cd k, WaveConst& W)
{
    const double ak = hypot(k.re, k.im);
    W.kr = k.re;
    W.ki = k.im;
    W.r2_small = (HANKEL_XS_F64 / ak) * (HANKEL_XS_F64 / ak);
    const cd xk = cdiv({HANKEL_XS_F64, 0.0}, k);  // XS / k
    W.ur = xk.re;
    W.ui = xk.im;
    const cd w = cmul(xk, xk);
    W.wr = w.re;
    W.wi = w.im;
    const cd sq = csqrt_(cdiv({2.0 / PI, 0.0}, k));  // sqrt(2/(pi k))
    const double c4 = 0.70710678118654752440;
    W.a0r = sq.re * c4 + sq.im * c4;  // * e^{-i pi/4} = (1 - i)/sqrt2
    W.a0i = sq.im * c4 - sq.re * c4;
    W.a1r = -sq.re * c4 + sq.im * c4;  // * e^{-3 i pi/4} = (-1 - i)/sqrt2
    W.a1i = -sq.im * c4 - sq.re * c4;
    const cd h = cscale(k, 0.5);
    W.hr = h.re;
    W.hi = h.im;
    const cd t = cmul(h, h);
    W.tr = t.re;
    W.ti = t.im;
    const cd lk = clog_(h);
    W.lkr = lk.re;
    W.lki = lk.im;
    const cd y1 = cdiv({-2.0 / PI, 0.0}, k);
    W.y1r = y1.re;
    W.y1i = y1.im;
}

__device__ void build_wave32(cd k, WaveConst32& W)
{
    const double ak = hypot(k.re, k.im);
    W.r2_small = (float)((HANKEL_XS_F32 / ak) * (HANKEL_XS_F32 / ak));
    const cd xk = cdiv({HANKEL_XS_F32, 0.0}, k);
    W.ur = (float)xk.re;
    W.ui = (float)xk.im;
    const cd w = cmul(xk, xk);
    W.wr = (float)w.re;
    W.wi = (float)w.im;
    const cd sq = csqrt_(cdiv({2.0 / PI, 0.0}, k));
    const double c4 = 0.70710678118654752440;
    W.a0r = (float)(sq.re * c4 + sq.im * c4);
    W.a0i = (float)(sq.im * c4 - sq.re * c4);
    W.a1r = (float)(-sq.re * c4 + sq.im * c4);
    W.a1i = (float)(-sq.im * c4 - sq.re * c4);
}

__global__ void k_domains(char* g, GeomLayout L)
{
    const int d = threadIdx.x;
    const GlobalIn G = *tab<GlobalIn>(g, L.glob_in);
    if (d >= G.n_dom) return;
    const DomIn* in = tab<DomIn>(g, L.dom_in);
    const cd k0 = {in[0].k[0], in[0].k[1]};
    const cd k = {in[d].k[0], in[d].k[1]};
    const cd r = cdiv(k, k0);
    const cd eps = cmul(r, r);
    // alpha = -i / k0 (Sec. 3.3) unless given
    const cd alpha = G.has_alpha ? cd{G.alpha[0], G.alpha[1]} : cdiv({0.0, -1.0}, k0);
    cd beta;
    if (G.has_beta)
        beta = {G.beta[0], G.beta[1]};
    else if (G.form == 0 || G.form == 3)
        beta = {-alpha.re, -alpha.im};
    else
        beta = {1.0, 0.0};
    const cd c = in[d].has_bm ? cd{in[d].bm[0], in[d].bm[1]} : cdiv(alpha, eps);
    DomConst D;
    D.k[0] = k.re;
    D.k[1] = k.im;
    D.eps[0] = eps.re;
    D.eps[1] = eps.im;
    D.c[0] = c.re;
    D.c[1] = c.im;
    D.beta[0] = beta.re;
    D.beta[1] = beta.im;
    D.cplx = (k.im != 0.0);
    D.pad = 0;
    tabw<DomConst>(g, L.dom)[d] = D;
    build_wave(k, tabw<WaveConst>(g, L.wave)[d]);
    build_wave32(k, tabw<WaveConst32>(g, L.wave32)[d]);
}

// ---------------------------------------------------------------------------
// Self term of the single-layer operator on a flat element at its midpoint
// (Sec. 7, the weak singularity): S_ii = (i/(2k)) int_0^{kh/2} H0(t) dt, the
// integral taken term by term from the ascending series of J0 and Y0.
// One lane per (element, domain on either side of it).
// ---------------------------------------------------------------------------
__device__ cd int_h0(cd z)
{
    const cd zh = cscale(z, 0.5);
    const cd q = cmul(zh, zh);
    const cd lz = clog_(zh);
    cd T = cscale(zh, 2.0);  // 2 (z/2)^{2m+1} (-1)^m / (m!)^2
    cd sj = {0.0, 0.0}, sj2 = {0.0, 0.0}, sh = {0.0, 0.0};
    double hm = 0.0;
    for (int m = 0; m < 200; ++m) {
        if (m > 0) {
            T = cscale(cmul(T, q), -1.0 / ((double)m * m));
            hm += 1.0 / m;
        }
        const double o = 2.0 * m + 1.0;
        const cd a = cscale(T, 1.0 / o);
        sj = cadd(sj, a);
        sj2 = cadd(sj2, cscale(T, 1.0 / (o * o)));
        sh = cadd(sh, cscale(a, hm));
        if (m > 3 && hypot(a.re, a.im) < 1e-18 * hypot(sj.re, sj.im)) break;
    }
    // int Y0 = (2/pi) [ (ln(z/2) + gamma) sum T/(2m+1) - sum T/(2m+1)^2 - sum H_m T/(2m+1) ]
    const cd ly = cmul({lz.re + EULER, lz.im}, sj);
    const cd iy = cscale({ly.re - sj2.re - sh.re, ly.im - sj2.im - sh.im}, 2.0 / PI);
    return {sj.re - iy.im, sj.im + iy.re};  // int J0 + i int Y0
}

__global__ void k_self_terms(char* g, GeomLayout L, int N, int n_dom)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= N) return;
    const ElemRec E = tab<ElemRec>(g, L.elem)[e];
    const int iface = tab<int>(g, L.elif)[e];
    const IfacePlan P = tab<IfacePlan>(g, L.iface)[iface];
    const DomConst* D = tab<DomConst>(g, L.dom);
    double2* S = tabw<double2>(g, L.self);
    for (int side = 0; side < 2; ++side) {
        const int d = side ? P.dr : P.dl;
        const cd k = {D[d].k[0], D[d].k[1]};
        const cd I = int_h0(cscale(k, 0.5 * E.h));
        const cd pre = cdiv({0.0, 0.5}, k);  // i / (2k)
        const cd s = cmul(pre, I);
        S[(size_t)d * N + e] = make_double2(s.re, s.im);
    }
}

// ---------------------------------------------------------------------------
// Fused assembly of one equation block (one side of an interface) against the
// elements of one interface.  Operators (eqs. (stmp)-(ddtmp)) of domain d
// between collocation point x_i and element j:
//   S  = (i/4)   sum_g w_g H0(k r_g)
//   D  = (ik/4)  sum_g w_g H1(k r_g) (r_g . n_j)/r_g
//   D* = -(ik/4) sum_g w_g H1(k r_g) (r_g . n_i)/r_g
//   N  = k^2 (n_i.n_j) S + (ik/4)[E(b_j) - E(a_j)],  E(p) = H1(k|x_i-p|) t_i.(x_i-p)/|x_i-p|
// (N by the identity d2G/dnx dny = k^2 (nx.ny) G - d2G/dtx dty, exact on a
// flat element; E at the shared end nodes is carried from element to element).
// Block entries (sigma = +1 if the normal leaves domain d, eps = eps_d):
//   standard row, scale s:  A[row, u_j] = s (delta/2 + sigma D),   A[row, w_j] = -s sigma eps S
//   Burton-Miller row, c:   A[row, u_j] = delta/2 + sigma (D + c N),
//                           A[row, w_j] = -sigma eps S + c (eps delta/2 - sigma eps D*)
// One lane per collocation row; the wave walks the source elements of its
// chunk in order (wave-uniform element data, coalesced column-major stores).
// ---------------------------------------------------------------------------
template <int Q, bool CPLX, bool BM>
__device__ __forceinline__ void assemble_side(const ElemRec* __restrict__ el, const GaussRec* __restrict__ gq,
                                              const WaveConst& W, const DomConst& Dm, int sg, int i,
                                              const ElemRec& Ei, int j0, int cnt, int q_rt, cd selfS,
                                              double2* __restrict__ A, size_t lda, float2* __restrict__ A32,
                                              size_t lda32, size_t row, int N)
{
    const int q = Q > 0 ? Q : q_rt;
    const cd k = {Dm.k[0], Dm.k[1]};
    const cd ik4 = {-0.25 * k.im, 0.25 * k.re};     // i k / 4
    const cd eps = {Dm.eps[0], Dm.eps[1]};
    const cd c = {Dm.c[0], Dm.c[1]};
    const cd beta = {Dm.beta[0], Dm.beta[1]};
    const double s = (double)sg;
    // per-block combination constants
    const cd cD = BM ? cd{s * ik4.re, s * ik4.im} : cscale(cmul(beta, ik4), s);  // multiplies sum D
    const cd iq = {0.0, 0.25};
    cd cS = cscale(cmul(eps, iq), -s);  // multiplies sum S (w column)
    if (!BM) cS = cmul(cS, beta);
    const cd cDs = cscale(cmul(cmul(c, eps), ik4), s);    // multiplies sum D* (note the minus signs cancel)
    const cd cNS = cscale(cmul(cmul(c, cmul(k, k)), iq), s);  // k^2 (n_i.n_j) S part of c sigma N
    const cd cNE = cscale(cmul(c, ik4), s);                   // end-point part of c sigma N
    const cd du = BM ? cd{0.5, 0.0} : cscale(beta, 0.5);      // jump term, u column
    const cd dw = cscale(cmul(c, eps), 0.5);                  // jump term, w column (BM only)

    const double xi = Ei.cx, yi = Ei.cy;
    cd Ea = {0.0, 0.0};
    if (BM) {
        const ElemRec& E0 = el[j0];
        const double dx = xi - E0.ax, dy = yi - E0.ay;
        const double r2 = dx * dx + dy * dy;
        const double r = sqrt(r2), rinv = 1.0 / r, sr = sqrt(rinv);
        const cd h1 = hankel1_only<CPLX>(W, r, r2, rinv, sr);
        Ea = cscale(h1, (Ei.tx * dx + Ei.ty * dy) * rinv);
    }
    for (int jj = 0; jj < cnt; ++jj) {
        const int j = j0 + jj;
        const ElemRec& Ej = el[j];
        cd sS = {0.0, 0.0}, sD = {0.0, 0.0}, sDs = {0.0, 0.0};
        const bool diag = (j == i);
        if (!diag) {
            const GaussRec& G = gq[j];
#pragma unroll ASM_GAUSS_UNROLL
            for (int g = 0; g < (Q > 0 ? Q : QMAX); ++g) {
                if (Q == 0 && g >= q) break;
                const double rx = xi - G.x[g], ry = yi - G.y[g];
                const double r2 = fma(rx, rx, ry * ry);
                const double r = sqrt(r2);
                const double rinv = 1.0 / r;
                const double sr = sqrt(rinv);
                cd h0, h1;
                hankel01<CPLX>(W, r, r2, rinv, sr, h0, h1);
                const double wg = G.w[g];
                sS.re = fma(wg, h0.re, sS.re);
                sS.im = fma(wg, h0.im, sS.im);
                const double wd = wg * (rx * Ej.nx + ry * Ej.ny) * rinv;
                sD.re = fma(wd, h1.re, sD.re);
                sD.im = fma(wd, h1.im, sD.im);
                if (BM) {
                    const double ws = wg * (rx * Ei.nx + ry * Ei.ny) * rinv;
                    sDs.re = fma(ws, h1.re, sDs.re);
                    sDs.im = fma(ws, h1.im, sDs.im);
                }
            }
        }
        cd au, aw;
        if (!diag) {
            au = cmul(cD, sD);
            aw = cmul(cS, sS);
        } else {
            // self term: D = D* = 0 on a flat element, S analytic; sS carries S / (i/4)
            const cd s4 = cdiv(selfS, iq);
            sS = s4;
            au = du;
            aw = cmul(cS, sS);
            if (BM) aw = cadd(aw, dw);
        }
        if (BM) {
            const double dxb = xi - Ej.bx, dyb = yi - Ej.by;
            const double r2 = dxb * dxb + dyb * dyb;
            const double r = sqrt(r2), rinv = 1.0 / r, sr = sqrt(rinv);
            const cd h1 = hankel1_only<CPLX>(W, r, r2, rinv, sr);
            const cd Eb = cscale(h1, (Ei.tx * dxb + Ei.ty * dyb) * rinv);
            const double ninj = Ei.nx * Ej.nx + Ei.ny * Ej.ny;
            au = cadd(au, cadd(cscale(cmul(cNS, sS), ninj), cmul(cNE, {Eb.re - Ea.re, Eb.im - Ea.im})));
            aw = cadd(aw, cmul(cDs, sDs));
            Ea = Eb;
        }
        A[row + (size_t)j * lda] = make_double2(au.re, au.im);
        A[row + (size_t)(N + j) * lda] = make_double2(aw.re, aw.im);
        if (A32) {
            A32[row + (size_t)j * lda32] = make_float2((float)au.re, (float)au.im);
            A32[row + (size_t)(N + j) * lda32] = make_float2((float)aw.re, (float)aw.im);
        }
    }
}

// A: the FP64 matrix; A32 (optional): its entries rounded to FP32, written in
// the same pass (the mixed path's inner products use it, its refinement
// residuals the FP64 matrix).
template <int Q, bool CPLX, bool BM>
__global__ __launch_bounds__(ROW_TILE, ASM_WAVES_PER_SIMD) void k_assemble_f64(const char* __restrict__ g, GeomLayout L,
                                                                                int N, int n_if, int q_rt,
                                                                                const int* __restrict__ tiles, int side,
                                                                                double2* __restrict__ A, size_t lda,
                                                                                float2* __restrict__ A32, size_t lda32)
{
    const Tile rt = tab<Tile>(g, L.rtiles)[tiles[blockIdx.x]];
    const Tile cc = tab<Tile>(g, L.cchunks)[blockIdx.y];
    const int li = threadIdx.x;
    if (li >= rt.count) return;
    const IfacePlan P = tab<IfacePlan>(g, L.iface)[rt.iface];
    const int d = side ? P.dr : P.dl;
    const int sg = tab<int>(g, L.sigma)[d * n_if + cc.iface];
    const int i = rt.start + li;
    const size_t row = (size_t)((side ? P.row_r : P.row_l) + (i - P.off));
    if (sg == 0) {
        for (int jj = 0; jj < cc.count; ++jj) {
            const int j = cc.start + jj;
            A[row + (size_t)j * lda] = make_double2(0.0, 0.0);
            A[row + (size_t)(N + j) * lda] = make_double2(0.0, 0.0);
            if (A32) {
                A32[row + (size_t)j * lda32] = make_float2(0.0f, 0.0f);
                A32[row + (size_t)(N + j) * lda32] = make_float2(0.0f, 0.0f);
            }
        }
        return;
    }
    const ElemRec* el = tab<ElemRec>(g, L.elem);
    const GaussRec* gq = tab<GaussRec>(g, L.gauss);
    const WaveConst& W = tab<WaveConst>(g, L.wave)[d];
    const DomConst Dm = tab<DomConst>(g, L.dom)[d];
    const ElemRec Ei = el[i];
    cd selfS = {0.0, 0.0};
    if (i >= cc.start && i < cc.start + cc.count) {
        const double2 sv = tab<double2>(g, L.self)[(size_t)d * N + i];
        selfS = {sv.x, sv.y};
    }
    assemble_side<Q, CPLX, BM>(el, gq, W, Dm, sg, i, Ei, cc.start, cc.count, q_rt, selfS, A, lda, A32, lda32, row,
                               N);
}


// ---------------------------------------------------------------------------
// FP32 assembly (precision path).  Entries are stored as complex64.  What
// decides the accuracy stays in FP64: the distance r and the phase k r (FP32
// would put an error of |k r| 6e-8 into every far entry), the ascending
// series for |k r| < 4, the self terms.  The amplitude polynomials of
// |k r| >= 4 (degree 6 in w), sin/cos of the phase reduced to [-pi, pi] and
// the quadrature sums run in FP32.
// ---------------------------------------------------------------------------
struct cf {
    float re, im;
};
__device__ __forceinline__ cf cmulf(cf a, cf b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }

// H0, H1 at k r with r given in FP64; result in FP32.
template <bool CPLX>
__device__ __forceinline__ void hankel01_mixed(const WaveConst& W64, const WaveConst32& W, double r, cf& h0, cf& h1)
{
    if (r * r < (double)W.r2_small) {
        const double r2 = r * r, rinv = 1.0 / r, sr = sqrt(rinv);
        cd a0, a1;
        hankel01<CPLX>(W64, r, r2, rinv, sr, a0, a1);
        h0 = {(float)a0.re, (float)a0.im};
        h1 = {(float)a1.re, (float)a1.im};
        return;
    }
    constexpr double TWO_PI = 6.283185307179586476925;
    constexpr double INV_TWO_PI = 0.159154943091895335769;
    const double ph = W64.kr * r;
    const double red = fma(-rint(ph * INV_TWO_PI), TWO_PI, ph);  // |red| <= pi (+ rounding)
    float sn, cs;
    sincosf((float)red, &sn, &cs);
    const float rf = (float)r;
    const float rinv = 1.0f / rf;
    const float rho = rinv * rinv;
    const float srinv = sqrtf(rinv);
    if (!CPLX) {
        const float w = W.wr * rho;
        const float m0 = poly_real(HANKEL_M0_F32, w), n0 = poly_real(HANKEL_N0_F32, w);
        const float m1 = poly_real(HANKEL_M1_F32, w), n1 = poly_real(HANKEL_N1_F32, w);
        const float u = W.ur * rinv;
        const cf e = {cs * srinv, sn * srinv};
        h0 = cmulf(cmulf(e, {W.a0r, W.a0i}), {m0, u * n0});
        h1 = cmulf(cmulf(e, {W.a1r, W.a1i}), {m1, u * n1});
    } else {
        const float x = W.wr * rho, y = W.wi * rho;
        const float R = 2.0f * x, S = fmaf(x, x, y * y);
        cf m0, n0, m1, n1;
        poly_cplx(HANKEL_M0_F32, x, y, R, S, m0.re, m0.im);
        poly_cplx(HANKEL_N0_F32, x, y, R, S, n0.re, n0.im);
        poly_cplx(HANKEL_M1_F32, x, y, R, S, m1.re, m1.im);
        poly_cplx(HANKEL_N1_F32, x, y, R, S, n1.re, n1.im);
        const cf u = {W.ur * rinv, W.ui * rinv};
        const cf un0 = cmulf(u, n0), un1 = cmulf(u, n1);
        const float damp = (float)exp(-W64.ki * r) * srinv;
        const cf e = {cs * damp, sn * damp};
        h0 = cmulf(cmulf(e, {W.a0r, W.a0i}), {m0.re - un0.im, m0.im + un0.re});
        h1 = cmulf(cmulf(e, {W.a1r, W.a1i}), {m1.re - un1.im, m1.im + un1.re});
    }
}

template <int Q, bool CPLX, bool BM>
__device__ __forceinline__ void assemble_side_f32(const ElemRec* __restrict__ el, const GaussRec* __restrict__ gq,
                                                  const WaveConst& W64, const WaveConst32& W, const DomConst& Dm,
                                                  int sg, int i, const ElemRec& Ei, int j0, int cnt, int q_rt,
                                                  cd selfS, float2* __restrict__ A, size_t lda, size_t row, int N)
{
    const int q = Q > 0 ? Q : q_rt;
    const cd k = {Dm.k[0], Dm.k[1]};
    const cd ik4 = {-0.25 * k.im, 0.25 * k.re};
    const cd eps = {Dm.eps[0], Dm.eps[1]};
    const cd c = {Dm.c[0], Dm.c[1]};
    const cd beta = {Dm.beta[0], Dm.beta[1]};
    const double s = (double)sg;
    const cd iq = {0.0, 0.25};
    const cd cD = BM ? cd{s * ik4.re, s * ik4.im} : cscale(cmul(beta, ik4), s);
    cd cS = cscale(cmul(eps, iq), -s);
    if (!BM) cS = cmul(cS, beta);
    const cd cDs = cscale(cmul(cmul(c, eps), ik4), s);
    const cd cNS = cscale(cmul(cmul(c, cmul(k, k)), iq), s);
    const cd cNE = cscale(cmul(c, ik4), s);
    const cd du = BM ? cd{0.5, 0.0} : cscale(beta, 0.5);
    const cd dw = cscale(cmul(c, eps), 0.5);
    const cf cDf = {(float)cD.re, (float)cD.im}, cSf = {(float)cS.re, (float)cS.im};
    const cf cDsf = {(float)cDs.re, (float)cDs.im}, cNSf = {(float)cNS.re, (float)cNS.im};
    const cf cNEf = {(float)cNE.re, (float)cNE.im};
    const double xi = Ei.cx, yi = Ei.cy;
    const float tix = (float)Ei.tx, tiy = (float)Ei.ty, nix = (float)Ei.nx, niy = (float)Ei.ny;
    cf Ea = {0.0f, 0.0f};
    if (BM) {
        const ElemRec& E0 = el[j0];
        const double dx = xi - E0.ax, dy = yi - E0.ay;
        const double r = sqrt(dx * dx + dy * dy);
        cf h0, h1;
        hankel01_mixed<CPLX>(W64, W, r, h0, h1);
        const float f = (float)((Ei.tx * dx + Ei.ty * dy) / r);
        Ea = {h1.re * f, h1.im * f};
    }
    for (int jj = 0; jj < cnt; ++jj) {
        const int j = j0 + jj;
        const ElemRec& Ej = el[j];
        cf sS = {0.0f, 0.0f}, sD = {0.0f, 0.0f}, sDs = {0.0f, 0.0f};
        const bool diag = (j == i);
        if (!diag) {
            const GaussRec& G = gq[j];
            const float njx = (float)Ej.nx, njy = (float)Ej.ny;
#pragma unroll ASM_GAUSS_UNROLL
            for (int g = 0; g < (Q > 0 ? Q : QMAX); ++g) {
                if (Q == 0 && g >= q) break;
                const double rx = xi - G.x[g], ry = yi - G.y[g];
                const double r = sqrt(fma(rx, rx, ry * ry));
                cf h0, h1;
                hankel01_mixed<CPLX>(W64, W, r, h0, h1);
                const float wg = (float)G.w[g];
                const float rxf = (float)rx, ryf = (float)ry, rif = (float)(1.0 / r);
                sS.re = fmaf(wg, h0.re, sS.re);
                sS.im = fmaf(wg, h0.im, sS.im);
                const float wd = wg * (rxf * njx + ryf * njy) * rif;
                sD.re = fmaf(wd, h1.re, sD.re);
                sD.im = fmaf(wd, h1.im, sD.im);
                if (BM) {
                    const float ws = wg * (rxf * nix + ryf * niy) * rif;
                    sDs.re = fmaf(ws, h1.re, sDs.re);
                    sDs.im = fmaf(ws, h1.im, sDs.im);
                }
            }
        }
        // combine in FP64 (few operations per entry), store FP32
        cd au, aw;
        cd sS64 = {(double)sS.re, (double)sS.im};
        if (!diag) {
            au = cmul(cD, {(double)sD.re, (double)sD.im});
            aw = cmul(cS, sS64);
        } else {
            sS64 = cdiv(selfS, iq);
            au = du;
            aw = cmul(cS, sS64);
            if (BM) aw = cadd(aw, dw);
        }
        if (BM) {
            const double dxb = xi - Ej.bx, dyb = yi - Ej.by;
            const double r = sqrt(dxb * dxb + dyb * dyb);
            cf h0, h1;
            hankel01_mixed<CPLX>(W64, W, r, h0, h1);
            const float f = (float)((Ei.tx * dxb + Ei.ty * dyb) / r);
            const cf Eb = {h1.re * f, h1.im * f};
            const double ninj = Ei.nx * Ej.nx + Ei.ny * Ej.ny;
            au = cadd(au, cadd(cscale(cmul(cNS, sS64), ninj),
                               cmul(cNE, {(double)Eb.re - (double)Ea.re, (double)Eb.im - (double)Ea.im})));
            aw = cadd(aw, cmul(cDs, {(double)sDs.re, (double)sDs.im}));
            Ea = Eb;
        }
        (void)cDf;
        (void)cSf;
        (void)cDsf;
        (void)cNSf;
        (void)cNEf;
        (void)tix;
        (void)tiy;
        A[row + (size_t)j * lda] = make_float2((float)au.re, (float)au.im);
        A[row + (size_t)(N + j) * lda] = make_float2((float)aw.re, (float)aw.im);
    }
}

template <int Q, bool CPLX, bool BM>
__global__ __launch_bounds__(ROW_TILE, ASM_WAVES_PER_SIMD) void k_assemble_f32(const char* __restrict__ g, GeomLayout L,
                                                                                int N, int n_if, int q_rt,
                                                                                const int* __restrict__ tiles, int side,
                                                                                float2* __restrict__ A, size_t lda)
{
    const Tile rt = tab<Tile>(g, L.rtiles)[tiles[blockIdx.x]];
    const Tile cc = tab<Tile>(g, L.cchunks)[blockIdx.y];
    const int li = threadIdx.x;
    if (li >= rt.count) return;
    const IfacePlan P = tab<IfacePlan>(g, L.iface)[rt.iface];
    const int d = side ? P.dr : P.dl;
    const int sg = tab<int>(g, L.sigma)[d * n_if + cc.iface];
    const int i = rt.start + li;
    const size_t row = (size_t)((side ? P.row_r : P.row_l) + (i - P.off));
    if (sg == 0) {
        for (int jj = 0; jj < cc.count; ++jj) {
            const int j = cc.start + jj;
            A[row + (size_t)j * lda] = make_float2(0.0f, 0.0f);
            A[row + (size_t)(N + j) * lda] = make_float2(0.0f, 0.0f);
        }
        return;
    }
    const ElemRec* el = tab<ElemRec>(g, L.elem);
    const GaussRec* gq = tab<GaussRec>(g, L.gauss);
    const WaveConst& W64 = tab<WaveConst>(g, L.wave)[d];
    const WaveConst32& W = tab<WaveConst32>(g, L.wave32)[d];
    const DomConst Dm = tab<DomConst>(g, L.dom)[d];
    const ElemRec Ei = el[i];
    cd selfS = {0.0, 0.0};
    if (i >= cc.start && i < cc.start + cc.count) {
        const double2 sv = tab<double2>(g, L.self)[(size_t)d * N + i];
        selfS = {sv.x, sv.y};
    }
    assemble_side_f32<Q, CPLX, BM>(el, gq, W64, W, Dm, sg, i, Ei, cc.start, cc.count, q_rt, selfS, A, lda, row, N);
}
}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_setup(char* g, const GeomLayout& L, int N, int n_dom, int q, hipStream_t s)
{
    hipLaunchKernelGGL(k_gauss_rule, dim3(1), dim3(64), 0, s, q, reinterpret_cast<double*>(g + L.gl));
    hipLaunchKernelGGL(k_domains, dim3(1), dim3(64), 0, s, g, L);
    hipLaunchKernelGGL(k_elements, dim3((N + 255) / 256), dim3(256), 0, s, g, L, N, q);
    hipLaunchKernelGGL(k_self_terms, dim3((N + 63) / 64), dim3(64), 0, s, g, L, N, n_dom);
    return hipGetLastError();
}

// One launch per variant (side of the interface, row type, complex wavenumber)
// over the row tiles of that variant; lists[v] / counts[v] are device / host.
template <class T2, bool F64, int Q>
void launch_variants(const char* g, const GeomLayout& L, int N, int n_if, int n_cchunks, int q,
                     const int* const* lists, const int* counts, T2* A, size_t lda, float2* A32, size_t lda32,
                     hipStream_t s)
{
    for (int v = 0; v < ASM_VARIANTS; ++v) {
        if (counts[v] == 0) continue;
        const int side = v >> 2 & 1, bm = v >> 1 & 1, cplx = v & 1;
        dim3 grid(counts[v], n_cchunks, 1);
#define BEM_ASM_LAUNCH(C_, B_)                                                                                  \
    if (cplx == C_ && bm == B_) {                                                                               \
        if constexpr (F64)                                                                                      \
            hipLaunchKernelGGL((k_assemble_f64<Q, C_, B_>), grid, dim3(ROW_TILE), 0, s, g, L, N, n_if, q, lists[v], \
                               side, reinterpret_cast<double2*>(A), lda, A32, lda32);                            \
        else                                                                                                    \
            hipLaunchKernelGGL((k_assemble_f32<Q, C_, B_>), grid, dim3(ROW_TILE), 0, s, g, L, N, n_if, q, lists[v], \
                               side, reinterpret_cast<float2*>(A), lda);                                         \
    }
        BEM_ASM_LAUNCH(false, false)
        BEM_ASM_LAUNCH(true, false)
        BEM_ASM_LAUNCH(false, true)
        BEM_ASM_LAUNCH(true, true)
#undef BEM_ASM_LAUNCH
    }
}

hipError_t launch_assemble_f64(const char* g, const GeomLayout& L, int N, int n_if, int n_cchunks, int q,
                               const int* const* lists, const int* counts, double2* A, size_t lda, float2* A32,
                               size_t lda32, hipStream_t s)
{
    if (q == 8)
        launch_variants<double2, true, 8>(g, L, N, n_if, n_cchunks, q, lists, counts, A, lda, A32, lda32, s);
    else if (q == 10)
        launch_variants<double2, true, 10>(g, L, N, n_if, n_cchunks, q, lists, counts, A, lda, A32, lda32, s);
    else
        launch_variants<double2, true, 0>(g, L, N, n_if, n_cchunks, q, lists, counts, A, lda, A32, lda32, s);
    return hipGetLastError();
}

hipError_t launch_assemble_f32(const char* g, const GeomLayout& L, int N, int n_if, int n_cchunks, int q,
                               const int* const* lists, const int* counts, float2* A, size_t lda, hipStream_t s)
{
    if (q == 8)
        launch_variants<float2, false, 8>(g, L, N, n_if, n_cchunks, q, lists, counts, A, lda, nullptr, 0, s);
    else if (q == 10)
        launch_variants<float2, false, 10>(g, L, N, n_if, n_cchunks, q, lists, counts, A, lda, nullptr, 0, s);
    else
        launch_variants<float2, false, 0>(g, L, N, n_if, n_cchunks, q, lists, counts, A, lda, nullptr, 0, s);
    return hipGetLastError();
}

}  // namespace bemk
