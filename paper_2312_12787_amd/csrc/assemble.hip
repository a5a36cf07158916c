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
// Assembly kernels: minimum waves per SIMD of the far-element and of the
// near-element launch (the latter reads its series coefficients by scalar
// loads) and Gauss points unrolled together (measured on gfx950, kite of 4096
// elements: one Gauss point at a time is 6 % faster than two in FP64, equal
// in FP32, and unrolling the near-element loop by 2 or 8 gains nothing; four
// waves per SIMD no faster than two; a third near-element wave makes the
// complex Burton-Miller variant spill).  The source elements per near-element
// workgroup, NEAR_PART, are set with the shared layout constants.
#ifndef ASM_FAR_WAVES
#define ASM_FAR_WAVES 2
#endif
#ifndef ASM_NEAR_WAVES
#define ASM_NEAR_WAVES 2
#endif
#ifndef ASM_GAUSS_UNROLL
#define ASM_GAUSS_UNROLL 1
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
    W.ampr = sq.re;
    W.ampi = sq.im;
    W.rs = HANKEL_XS_F64 / ak;
    W.rs32 = HANKEL_XS_F32 / ak;
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
    W.ampr = (float)sq.re;
    W.ampi = (float)sq.im;
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
// One lane per collocation row (a workgroup: ROW_TILE rows against a chunk of
// COL_CHUNK source elements).  The chunk's Gauss points and element data are
// staged in LDS once per workgroup; each wave then splits the chunk by a
// wave-uniform test: an element whose every point lies at least XS/|k| from
// all of the wave's collocation points is "far" and takes the large-argument
// Hankel form alone (hankel01_far: no series, no per-lane branch); the rest
// (the element itself, its neighbours, close parts of a non-convex curve)
// take the general per-lane evaluation.  The far elements are walked first,
// the near ones after, so that the series coefficients are not live in the
// far loop.  Stores are coalesced column-major (consecutive lanes = rows).
// ---------------------------------------------------------------------------
static_assert(XS_SERIES_F64 == HANKEL_XS_F64 && XS_SERIES_F32 == HANKEL_XS_F32,
              "the host's near-pair lists use the series radii of the device evaluator");

struct GaussL {
    double x, y, w, pad;
};
struct ElemL {
    double nx, ny, ax, ay, bx, by, cx, cy, hh, pad;  // normal, nodes, midpoint, h/2
};

// Per-block combination constants of one equation block (see the entries above).
struct BlockConst {
    cd cD, cS, cDs, cNS, cNE, du, dw, iq;
};

template <bool BM>
__device__ __forceinline__ BlockConst block_const(const DomConst& Dm, int sg)
{
    const cd k = {Dm.k[0], Dm.k[1]};
    const cd ik4 = {-0.25 * k.im, 0.25 * k.re};  // i k / 4
    const cd eps = {Dm.eps[0], Dm.eps[1]};
    const cd c = {Dm.c[0], Dm.c[1]};
    const cd beta = {Dm.beta[0], Dm.beta[1]};
    const double s = (double)sg;
    BlockConst B;
    B.iq = {0.0, 0.25};
    B.cD = BM ? cd{s * ik4.re, s * ik4.im} : cscale(cmul(beta, ik4), s);  // multiplies sum D
    B.cS = cscale(cmul(eps, B.iq), -s);                                   // multiplies sum S (w column)
    if (!BM) B.cS = cmul(B.cS, beta);
    B.cDs = cscale(cmul(cmul(c, eps), ik4), s);            // multiplies sum D* (the minus signs cancel)
    B.cNS = cscale(cmul(cmul(c, cmul(k, k)), B.iq), s);    // k^2 (n_i.n_j) S part of c sigma N
    B.cNE = cscale(cmul(c, ik4), s);                       // end-point part of c sigma N
    B.du = BM ? cd{0.5, 0.0} : cscale(beta, 0.5);          // jump term, u column
    B.dw = cscale(cmul(c, eps), 0.5);                      // jump term, w column (BM only)
    return B;
}

// End-point value E(p) = H1(k|x_i - p|) t_i.(x_i - p)/|x_i - p| (without the ik/4).
template <bool CPLX, bool FAR>
__device__ __forceinline__ cd end_value(const WaveConst& W, double xi, double yi, double tix, double tiy, double px,
                                        double py)
{
    const double dx = xi - px, dy = yi - py;
    cd h0, h1;
    double rinv;
    if (FAR) {
        rinv = hankel01_far<CPLX, false>(W, dx, dy, h0, h1);
    } else {
        const double r2 = dx * dx + dy * dy;
        double r;
        sqrt_rsqrt(r2, r, rinv);
        h1 = hankel1_only<CPLX, true>(W, r, r2, rinv, rsqrt_nr(r));
    }
    return cscale(h1, (tix * dx + tiy * dy) * rinv);
}

// One matrix entry pair (u column, w column) of row i against element j.
template <int Q, bool CPLX, bool BM, bool FAR>
__device__ __forceinline__ void element_entries(const WaveConst& W, const BlockConst& B, const ElemRec& Ei,
                                                const ElemL& Ej, const GaussL* __restrict__ gp, int q_rt,
                                                bool diag, cd selfS, cd& Ea, bool carry, cd& au, cd& aw)
{
    const int q = Q > 0 ? Q : q_rt;
    const double xi = Ei.cx, yi = Ei.cy;
    cd sS = {0.0, 0.0}, sD = {0.0, 0.0}, sDs = {0.0, 0.0};
    if (FAR || !diag) {
#pragma unroll ASM_GAUSS_UNROLL
        for (int g = 0; g < (Q > 0 ? Q : QMAX); ++g) {
            if (Q == 0 && g >= q) break;
            const GaussL P = gp[g];
            const double rx = xi - P.x, ry = yi - P.y;
            cd h0, h1;
            double rinv;
            if (FAR) {
                rinv = hankel01_far<CPLX, true>(W, rx, ry, h0, h1);
            } else {
                const double r2 = fma(rx, rx, ry * ry);
                double r;
                sqrt_rsqrt(r2, r, rinv);
                hankel01<CPLX, true>(W, r, r2, rinv, rsqrt_nr(r), h0, h1);
            }
            sS.re = fma(P.w, h0.re, sS.re);
            sS.im = fma(P.w, h0.im, sS.im);
            const double wr = P.w * rinv;
            const double wd = wr * fma(rx, Ej.nx, ry * Ej.ny);
            sD.re = fma(wd, h1.re, sD.re);
            sD.im = fma(wd, h1.im, sD.im);
            if (BM) {
                const double ws = wr * fma(rx, Ei.nx, ry * Ei.ny);
                sDs.re = fma(ws, h1.re, sDs.re);
                sDs.im = fma(ws, h1.im, sDs.im);
            }
        }
    }
    if (FAR || !diag) {
        au = cmul(B.cD, sD);
        aw = cmul(B.cS, sS);
    } else {
        // self term: D = D* = 0 on a flat element, S analytic; sS carries S / (i/4)
        sS = cdiv(selfS, B.iq);
        au = B.du;
        aw = cmul(B.cS, sS);
        if (BM) aw = cadd(aw, B.dw);
    }
    if (BM) {
        if (!carry) Ea = end_value<CPLX, FAR>(W, xi, yi, Ei.tx, Ei.ty, Ej.ax, Ej.ay);
        const cd Eb = end_value<CPLX, FAR>(W, xi, yi, Ei.tx, Ei.ty, Ej.bx, Ej.by);
        const double ninj = Ei.nx * Ej.nx + Ei.ny * Ej.ny;
        au = cadd(au, cadd(cscale(cmul(B.cNS, sS), ninj), cmul(B.cNE, {Eb.re - Ea.re, Eb.im - Ea.im})));
        aw = cadd(aw, cmul(B.cDs, sDs));
        Ea = Eb;  // E(b_j) = E(a_{j+1}): carried to the next element of the same walk
    }
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

template <bool CPLX>
__device__ __forceinline__ void hankel_far32_body(const WaveConst& W64, const WaveConst32& W, double r, float& h0r,
                                                  float& h0i, float& h1r, float& h1i);

// H0, H1 at k r with r given in FP64; result in FP32.
template <bool CPLX, bool MEM = false>
__device__ __forceinline__ void hankel01_mixed(const WaveConst& W64, const WaveConst32& W, double r, cf& h0, cf& h1)
{
    // one write of h0, h1 after the join (as in hankel01)
    float h0r, h0i, h1r, h1i;
    if (r * r < (double)W.r2_small) {
        const double r2 = r * r, rinv = 1.0 / r, sr = sqrt(rinv);
        cd a0, a1;
        hankel01<CPLX, MEM>(W64, r, r2, rinv, sr, a0, a1);
        h0r = (float)a0.re;
        h0i = (float)a0.im;
        h1r = (float)a1.re;
        h1i = (float)a1.im;
    } else {
        hankel_far32_body<CPLX>(W64, W, r, h0r, h0i, h1r, h1i);
    }
    h0 = {h0r, h0i};
    h1 = {h1r, h1i};
}

// The large-argument branch of hankel01_mixed.
template <bool CPLX>
__device__ __forceinline__ void hankel_far32_body(const WaveConst& W64, const WaveConst32& W, double r, float& h0r,
                                                  float& h0i, float& h1r, float& h1i)
{
    cf h0, h1;
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
    h0r = h0.re;
    h0i = h0.im;
    h1r = h1.re;
    h1i = h1.im;
}

// FP32 large-argument form for |k r| >= XS_F32 (no series, no per-lane
// branch): distance, phase and its reduction by pi/2 in FP64, the reduced
// angle's sine and cosine, the amplitude polynomials and the products in FP32.
// Returns 1/r.
__device__ __forceinline__ void sincos_cw32(double x, float& s, float& c)
{
    constexpr double TWO_OVER_PI = 0x1.45f306dc9c883p-1;
    constexpr double P1 = 0x1.921fb54442d18p+0;
    constexpr double P2 = 0x1.1a62633145c07p-54;
    const double n = rint(x * TWO_OVER_PI);
    const float t = (float)fma(-n, P2, fma(-n, P1, x));
    const float u = t * t;
    // Taylor series on |t| <= pi/4: sin to t^9 (truncation < 2e-9), cos to t^10 (< 2e-10)
    const float st = fmaf(t * u, fmaf(u, fmaf(u, fmaf(u, 1.0f / 362880.0f, -1.0f / 5040.0f), 1.0f / 120.0f),
                                      -1.0f / 6.0f), t);
    const float ct = fmaf(u, fmaf(u, fmaf(u, fmaf(u, fmaf(u, -1.0f / 3628800.0f, 1.0f / 40320.0f), -1.0f / 720.0f),
                                          1.0f / 24.0f), -0.5f), 1.0f);
    const unsigned q = (unsigned)(int)n;
    const float a = (q & 1u) ? ct : st;
    const float b = (q & 1u) ? st : ct;
    s = __uint_as_float(__float_as_uint(a) ^ ((q & 2u) << 30));
    c = __uint_as_float(__float_as_uint(b) ^ (((q + 1u) & 2u) << 30));
}

template <bool CPLX, bool WANT_H0>
__device__ __forceinline__ float hankel01_far32(const WaveConst& W64, const WaveConst32& W, double rx, double ry,
                                                cf& h0, cf& h1)
{
    constexpr double PI_4 = 0x1.921fb54442d18p-1;
    const double r2 = fma(rx, rx, ry * ry);
    double r, rinv;
    sqrt_rsqrt(r2, r, rinv);
    float sn, cs;
    sincos_cw32(fma(W64.kr, r, -PI_4), sn, cs);
    const float ri = (float)rinv;
    const float sr = __builtin_amdgcn_rsqf((float)r);
    const float rho = ri * ri;
    if (!CPLX) {
        const float w = W.wr * rho;
        const float u = W.ur * ri;
        const float a = W.ampr * sr;
        const float er = cs * a, ei = sn * a;
        const float m1 = poly_real(HANKEL_M1_F32, w), un1 = u * poly_real(HANKEL_N1_F32, w);
        h1 = {fmaf(er, un1, ei * m1), fmaf(ei, un1, -er * m1)};
        if (WANT_H0) {
            const float m0 = poly_real(HANKEL_M0_F32, w), un0 = u * poly_real(HANKEL_N0_F32, w);
            h0 = {fmaf(er, m0, -ei * un0), fmaf(er, un0, ei * m0)};
        }
    } else {
        const float x = W.wr * rho, y = W.wi * rho;
        const float R = 2.0f * x, S = fmaf(x, x, y * y);
        const cf u = {W.ur * ri, W.ui * ri};
        const float damp = expf((float)(-W64.ki * r)) * sr;
        const cf e = cmulf({cs * damp, sn * damp}, {W.ampr, W.ampi});
        cf m1, n1;
        poly_cplx(HANKEL_M1_F32, x, y, R, S, m1.re, m1.im);
        poly_cplx(HANKEL_N1_F32, x, y, R, S, n1.re, n1.im);
        const cf un1 = cmulf(u, n1);
        h1 = cmulf(e, {m1.im + un1.re, un1.im - m1.re});
        if (WANT_H0) {
            cf m0, n0;
            poly_cplx(HANKEL_M0_F32, x, y, R, S, m0.re, m0.im);
            poly_cplx(HANKEL_N0_F32, x, y, R, S, n0.re, n0.im);
            const cf un0 = cmulf(u, n0);
            h0 = cmulf(e, {m0.re - un0.im, m0.im + un0.re});
        }
    }
    return ri;
}

template <bool CPLX, bool FAR>
__device__ __forceinline__ cf end_value32(const WaveConst& W64, const WaveConst32& W, double xi, double yi, double tix,
                                          double tiy, double px, double py)
{
    const double dx = xi - px, dy = yi - py;
    cf h0, h1;
    double rinv;
    if (FAR) {
        rinv = hankel01_far32<CPLX, false>(W64, W, dx, dy, h0, h1);
    } else {
        const double r = sqrt(dx * dx + dy * dy);
        hankel01_mixed<CPLX, true>(W64, W, r, h0, h1);
        rinv = 1.0 / r;
    }
    const float f = (float)((tix * dx + tiy * dy) * rinv);
    return {h1.re * f, h1.im * f};
}

// FP32 sums over the Gauss points; the combination into entries runs in FP64.
template <int Q, bool CPLX, bool BM, bool FAR>
__device__ __forceinline__ void element_entries_f32(const WaveConst& W64, const WaveConst32& W, const BlockConst& B,
                                                    const ElemRec& Ei, const ElemL& Ej, const GaussL* __restrict__ gp,
                                                    int q_rt, bool diag, cd selfS, cf& Ea, bool carry, cd& au,
                                                    cd& aw)
{
    const int q = Q > 0 ? Q : q_rt;
    const double xi = Ei.cx, yi = Ei.cy;
    const float njx = (float)Ej.nx, njy = (float)Ej.ny, nix = (float)Ei.nx, niy = (float)Ei.ny;
    cf sS = {0.0f, 0.0f}, sD = {0.0f, 0.0f}, sDs = {0.0f, 0.0f};
    if (FAR || !diag) {
#pragma unroll ASM_GAUSS_UNROLL
        for (int g = 0; g < (Q > 0 ? Q : QMAX); ++g) {
            if (Q == 0 && g >= q) break;
            const GaussL P = gp[g];
            const double rx = xi - P.x, ry = yi - P.y;
            cf h0, h1;
            float ri;
            if (FAR) {
                ri = hankel01_far32<CPLX, true>(W64, W, rx, ry, h0, h1);
            } else {
                const double r = sqrt(fma(rx, rx, ry * ry));
                hankel01_mixed<CPLX, true>(W64, W, r, h0, h1);
                ri = (float)(1.0 / r);
            }
            const float wg = (float)P.w;
            sS.re = fmaf(wg, h0.re, sS.re);
            sS.im = fmaf(wg, h0.im, sS.im);
            const float rxf = (float)rx, ryf = (float)ry, wr = wg * ri;
            const float wd = wr * fmaf(rxf, njx, ryf * njy);
            sD.re = fmaf(wd, h1.re, sD.re);
            sD.im = fmaf(wd, h1.im, sD.im);
            if (BM) {
                const float ws = wr * fmaf(rxf, nix, ryf * niy);
                sDs.re = fmaf(ws, h1.re, sDs.re);
                sDs.im = fmaf(ws, h1.im, sDs.im);
            }
        }
    }
    cd sS64 = {(double)sS.re, (double)sS.im};
    if (FAR || !diag) {
        au = cmul(B.cD, {(double)sD.re, (double)sD.im});
        aw = cmul(B.cS, sS64);
    } else {
        sS64 = cdiv(selfS, B.iq);
        au = B.du;
        aw = cmul(B.cS, sS64);
        if (BM) aw = cadd(aw, B.dw);
    }
    if (BM) {
        if (!carry) Ea = end_value32<CPLX, FAR>(W64, W, xi, yi, Ei.tx, Ei.ty, Ej.ax, Ej.ay);
        const cf Eb = end_value32<CPLX, FAR>(W64, W, xi, yi, Ei.tx, Ei.ty, Ej.bx, Ej.by);
        const double ninj = Ei.nx * Ej.nx + Ei.ny * Ej.ny;
        au = cadd(au, cadd(cscale(cmul(B.cNS, sS64), ninj),
                           cmul(B.cNE, {(double)Eb.re - (double)Ea.re, (double)Eb.im - (double)Ea.im})));
        aw = cadd(aw, cmul(B.cDs, {(double)sDs.re, (double)sDs.im}));
        Ea = Eb;
    }
}

// ---------------------------------------------------------------------------
// The assembly kernels.  F32 = false: FP64 entries into A (double2) and, when
// A32 is given, the same entries rounded to FP32 into A32 in the same pass
// (the mixed path's inner products use that copy, its refinement residuals
// the FP64 matrix).  F32 = true: FP32 entries into A (float2).
// ---------------------------------------------------------------------------
// sub < 0: the workgroup's ROW_TILE threads cover the row tile and share the
// staged chunk (far launch).  sub >= 0: this wave alone covers rows
// [64 sub, 64 sub + 64) of the tile and stages its own part of the chunk in
// its own gp / ell (near launch: one list item per wave, so that waves whose
// rows have no near element are not launched at all).  Every wave of the
// workgroup reaches the one barrier, item or not (act).
template <int Q, bool CPLX, bool BM, bool F32, bool NEAR>
__device__ __forceinline__ void assemble_chunk(const char* __restrict__ g, const GeomLayout& L, int N, int n_if,
                                               int q_rt, int tile, int sub, int chunk, int part, int side, void* Av,
                                               size_t lda, float2* __restrict__ A32, size_t lda32,
                                               GaussL* __restrict__ gp, ElemL* __restrict__ ell, bool act)
{
    static_assert(COL_CHUNK <= 32, "the near-element mask is one 32-bit word");
    constexpr int QS = Q > 0 ? Q : QMAX;
    const int nst = sub < 0 ? ROW_TILE : 64;
    const int li_st = sub < 0 ? (int)threadIdx.x : (int)(threadIdx.x & 63);
    const int li = sub < 0 ? (int)threadIdx.x : sub * 64 + (int)(threadIdx.x & 63);
    Tile rt{}, cc{};
    int d = 0, sg = 0;
    IfacePlan P{};
    if (act) {
        rt = tab<Tile>(g, L.rtiles)[tile];
        cc = tab<Tile>(g, L.cchunks)[chunk];
        if (part >= 0) {  // near launch: NEAR_PART elements of the chunk
            cc.start += part * NEAR_PART;
            cc.count = min(NEAR_PART, cc.count - part * NEAR_PART);
        }
        P = tab<IfacePlan>(g, L.iface)[rt.iface];
        d = side ? P.dr : P.dl;
        sg = tab<int>(g, L.sigma)[d * n_if + cc.iface];
    }
    const int i = rt.start + li;
    const size_t row = (size_t)((side ? P.row_r : P.row_l) + (i - P.off));
    const int cnt = cc.count;
    auto store = [&](int j, cd au, cd aw) {
        if (F32) {
            float2* A = static_cast<float2*>(Av);
            A[row + (size_t)j * lda] = make_float2((float)au.re, (float)au.im);
            A[row + (size_t)(N + j) * lda] = make_float2((float)aw.re, (float)aw.im);
        } else {
            double2* A = static_cast<double2*>(Av);
            A[row + (size_t)j * lda] = make_double2(au.re, au.im);
            A[row + (size_t)(N + j) * lda] = make_double2(aw.re, aw.im);
            if (A32) {
                A32[row + (size_t)j * lda32] = make_float2((float)au.re, (float)au.im);
                A32[row + (size_t)(N + j) * lda32] = make_float2((float)aw.re, (float)aw.im);
            }
        }
    };
    if (!NEAR && sg == 0) {  // uniform over the workgroup; the far launch writes the zero block
        if (li >= rt.count) return;
        for (int jj = 0; jj < cnt; ++jj) store(cc.start + jj, {0.0, 0.0}, {0.0, 0.0});
        return;
    }
    act = act && sg != 0;
    // stage the chunk: Gauss points (x, y, weight) and element data
    if (act) {
        const int q = Q > 0 ? Q : q_rt;
        const GaussRec* gq = tab<GaussRec>(g, L.gauss);
        for (int t = li_st; t < cnt * q; t += nst) {
            const int e = t / q, gg = t - e * q;
            const GaussRec& G = gq[cc.start + e];
            gp[e * QS + gg] = GaussL{G.x[gg], G.y[gg], G.w[gg], 0.0};
        }
        const ElemRec* el = tab<ElemRec>(g, L.elem);
        for (int t = li_st; t < cnt; t += nst) {
            const ElemRec& E = el[cc.start + t];
            ell[t] = ElemL{E.nx, E.ny, E.ax, E.ay, E.bx, E.by, E.cx, E.cy, 0.5 * E.h, 0.0};
        }
    }
    __syncthreads();
    if (!act || li >= rt.count) return;
    const WaveConst& W = tab<WaveConst>(g, L.wave)[d];
    const DomConst Dm = tab<DomConst>(g, L.dom)[d];
    const ElemRec Ei = tab<ElemRec>(g, L.elem)[i];
    const BlockConst B = block_const<BM>(Dm, sg);
    cd selfS = {0.0, 0.0};
    if (i >= cc.start && i < cc.start + cnt) {
        const double2 sv = tab<double2>(g, L.self)[(size_t)d * N + i];
        selfS = {sv.x, sv.y};
    }
    // near mask: bit jj when some collocation point of this wave lies within
    // the series radius of a point of element jj (the element's points lie
    // within h/2 of its midpoint).  The near launch widens the radius by a
    // relative 1e-9, so that no element escapes both launches through a
    // rounding difference; an element both take is written by the near
    // launch, which runs second.
    const double rs = (F32 ? W.rs32 : W.rs) * (NEAR ? 1.0 + 1e-9 : 1.0);
    unsigned nearm = 0;
    for (int jj = 0; jj < cnt; ++jj) {
        const double dx = Ei.cx - ell[jj].cx, dy = Ei.cy - ell[jj].cy;
        const double lim = rs + ell[jj].hh;
        if (__builtin_amdgcn_ballot_w64(fma(dx, dx, dy * dy) < lim * lim) != 0) nearm |= 1u << jj;
    }
    const unsigned all = cnt >= 32 ? 0xffffffffu : (1u << cnt) - 1u;
    if (F32) {
        const WaveConst32& W32 = tab<WaveConst32>(g, L.wave32)[d];
        cf Ea = {0.0f, 0.0f};
        int prev = -2;
        for (unsigned m = NEAR ? 0u : all & ~nearm; m != 0; m &= m - 1) {
            const int jj = __builtin_ctz(m);
            cd au, aw;
            element_entries_f32<Q, CPLX, BM, true>(W, W32, B, Ei, ell[jj], gp + jj * QS, q_rt, false, selfS, Ea,
                                                   jj == prev + 1, au, aw);
            prev = jj;
            store(cc.start + jj, au, aw);
        }
        prev = -2;
        for (unsigned m = NEAR ? nearm : 0u; m != 0; m &= m - 1) {
            const int jj = __builtin_ctz(m);
            const int j = cc.start + jj;
            cd au, aw;
            element_entries_f32<Q, CPLX, BM, false>(W, W32, B, Ei, ell[jj], gp + jj * QS, q_rt, j == i, selfS, Ea,
                                                    jj == prev + 1, au, aw);
            prev = jj;
            store(j, au, aw);
        }
    } else {
        cd Ea = {0.0, 0.0};
        int prev = -2;
        for (unsigned m = NEAR ? 0u : all & ~nearm; m != 0; m &= m - 1) {
            const int jj = __builtin_ctz(m);
            cd au, aw;
            element_entries<Q, CPLX, BM, true>(W, B, Ei, ell[jj], gp + jj * QS, q_rt, false, selfS, Ea,
                                               jj == prev + 1, au, aw);
            prev = jj;
            store(cc.start + jj, au, aw);
        }
        prev = -2;
        for (unsigned m = NEAR ? nearm : 0u; m != 0; m &= m - 1) {
            const int jj = __builtin_ctz(m);
            const int j = cc.start + jj;
            cd au, aw;
            element_entries<Q, CPLX, BM, false>(W, B, Ei, ell[jj], gp + jj * QS, q_rt, j == i, selfS, Ea,
                                                jj == prev + 1, au, aw);
            prev = jj;
            store(j, au, aw);
        }
    }
}

// Far elements (the bulk; no series code, so two waves fit per SIMD) over the
// grid (row tiles of the variant) x (column chunks), and near elements (the
// general per-lane evaluation) over the variant's list of (row tile and its
// 64-row wave, column chunk, part of NEAR_PART elements) items whose bounding
// boxes come within the series radius, one item per wave.
template <int Q, bool CPLX, bool BM>
__global__ __launch_bounds__(ROW_TILE, ASM_FAR_WAVES) void k_assemble_f64(const char* __restrict__ g, GeomLayout L,
                                                                           int N, int n_if, int q_rt,
                                                                           const int* __restrict__ tiles, int side,
                                                                           double2* __restrict__ A, size_t lda,
                                                                           float2* __restrict__ A32, size_t lda32)
{
    __shared__ GaussL gp[COL_CHUNK * (Q > 0 ? Q : QMAX)];
    __shared__ ElemL ell[COL_CHUNK];
    assemble_chunk<Q, CPLX, BM, false, false>(g, L, N, n_if, q_rt, tiles[blockIdx.x], -1, blockIdx.y, -1, side, A, lda,
                                              A32, lda32, gp, ell, true);
}

constexpr int NEAR_WAVES = ROW_TILE / 64;  // list items per near-element workgroup
static_assert(NEAR_WAVES == 4, "a near item packs the wave of its row tile in two bits");

// The list item of this wave: (row tile * 4 + wave of the tile, chunk, part).
__device__ __forceinline__ bool near_item(const int* __restrict__ items, int count, int& tile, int& sub, int& chunk,
                                          int& part)
{
    const int k = blockIdx.x * NEAR_WAVES + (int)(threadIdx.x >> 6);
    if (k >= count) return false;
    const int tw = items[3 * k];
    tile = tw >> 2;
    sub = tw & 3;
    chunk = items[3 * k + 1];
    part = items[3 * k + 2];
    return true;
}

template <int Q, bool CPLX, bool BM>
__global__ __launch_bounds__(ROW_TILE, ASM_NEAR_WAVES) void k_assemble_near_f64(const char* __restrict__ g, GeomLayout L, int N,
                                                                   int n_if, int q_rt, const int* __restrict__ items,
                                                                   int count, int side, double2* __restrict__ A,
                                                                   size_t lda, float2* __restrict__ A32, size_t lda32)
{
    __shared__ GaussL gp[NEAR_WAVES][NEAR_PART * (Q > 0 ? Q : QMAX)];
    __shared__ ElemL ell[NEAR_WAVES][NEAR_PART];
    int tile = 0, sub = 0, chunk = 0, part = 0;
    const bool act = near_item(items, count, tile, sub, chunk, part);
    const int w = threadIdx.x >> 6;
    assemble_chunk<Q, CPLX, BM, false, true>(g, L, N, n_if, q_rt, tile, sub, chunk, part, side, A, lda, A32, lda32,
                                             gp[w], ell[w], act);
}

template <int Q, bool CPLX, bool BM>
__global__ __launch_bounds__(ROW_TILE, ASM_FAR_WAVES) void k_assemble_f32(const char* __restrict__ g, GeomLayout L,
                                                                           int N, int n_if, int q_rt,
                                                                           const int* __restrict__ tiles, int side,
                                                                           float2* __restrict__ A, size_t lda)
{
    __shared__ GaussL gp[COL_CHUNK * (Q > 0 ? Q : QMAX)];
    __shared__ ElemL ell[COL_CHUNK];
    assemble_chunk<Q, CPLX, BM, true, false>(g, L, N, n_if, q_rt, tiles[blockIdx.x], -1, blockIdx.y, -1, side, A, lda,
                                             nullptr, 0, gp, ell, true);
}

template <int Q, bool CPLX, bool BM>
__global__ __launch_bounds__(ROW_TILE, ASM_NEAR_WAVES) void k_assemble_near_f32(const char* __restrict__ g, GeomLayout L, int N,
                                                                   int n_if, int q_rt, const int* __restrict__ items,
                                                                   int count, int side, float2* __restrict__ A,
                                                                   size_t lda)
{
    __shared__ GaussL gp[NEAR_WAVES][NEAR_PART * (Q > 0 ? Q : QMAX)];
    __shared__ ElemL ell[NEAR_WAVES][NEAR_PART];
    int tile = 0, sub = 0, chunk = 0, part = 0;
    const bool act = near_item(items, count, tile, sub, chunk, part);
    const int w = threadIdx.x >> 6;
    assemble_chunk<Q, CPLX, BM, true, true>(g, L, N, n_if, q_rt, tile, sub, chunk, part, side, A, lda, nullptr, 0,
                                            gp[w], ell[w], act);
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
                     const int* const* lists, const int* counts, const int* const* pairs, const int* pair_counts,
                     T2* A, size_t lda, float2* A32, size_t lda32, hipStream_t s0, hipStream_t s1)
{
    int k = 0;  // variants write disjoint rows: alternate them over the two streams
    for (int v = 0; v < ASM_VARIANTS; ++v) {
        if (counts[v] == 0) continue;
        const hipStream_t s = (k++ & 1) ? s1 : s0;
        const int side = v >> 2 & 1, bm = v >> 1 & 1, cplx = v & 1;
        const dim3 grid(counts[v], n_cchunks, 1), ngrid((pair_counts[v] + NEAR_WAVES - 1) / NEAR_WAVES, 1, 1);
#define BEM_ASM_LAUNCH(C_, B_)                                                                                    \
    if (cplx == C_ && bm == B_) {                                                                                 \
        if constexpr (F64) {                                                                                      \
            hipLaunchKernelGGL((k_assemble_f64<Q, C_, B_>), grid, dim3(ROW_TILE), 0, s, g, L, N, n_if, q, lists[v],   \
                               side, reinterpret_cast<double2*>(A), lda, A32, lda32);                              \
            if (pair_counts[v] > 0)                                                                               \
                hipLaunchKernelGGL((k_assemble_near_f64<Q, C_, B_>), ngrid, dim3(ROW_TILE), 0, s, g, L, N, n_if, q,   \
                                   pairs[v], pair_counts[v], side, reinterpret_cast<double2*>(A), lda, A32, lda32);\
        } else {                                                                                                  \
            hipLaunchKernelGGL((k_assemble_f32<Q, C_, B_>), grid, dim3(ROW_TILE), 0, s, g, L, N, n_if, q, lists[v],   \
                               side, reinterpret_cast<float2*>(A), lda);                                           \
            if (pair_counts[v] > 0)                                                                               \
                hipLaunchKernelGGL((k_assemble_near_f32<Q, C_, B_>), ngrid, dim3(ROW_TILE), 0, s, g, L, N, n_if, q,   \
                                   pairs[v], pair_counts[v], side, reinterpret_cast<float2*>(A), lda);             \
        }                                                                                                         \
    }
        BEM_ASM_LAUNCH(false, false)
        BEM_ASM_LAUNCH(true, false)
        BEM_ASM_LAUNCH(false, true)
        BEM_ASM_LAUNCH(true, true)
#undef BEM_ASM_LAUNCH
    }
}

hipError_t launch_assemble_f64(const char* g, const GeomLayout& L, int N, int n_if, int n_cchunks, int q,
                               const int* const* lists, const int* counts, const int* const* pairs,
                               const int* pair_counts, double2* A, size_t lda, float2* A32, size_t lda32,
                               hipStream_t s, hipStream_t s1)
{
    if (q == 8)
        launch_variants<double2, true, 8>(g, L, N, n_if, n_cchunks, q, lists, counts, pairs, pair_counts, A, lda, A32,
                                          lda32, s, s1);
    else if (q == 10)
        launch_variants<double2, true, 10>(g, L, N, n_if, n_cchunks, q, lists, counts, pairs, pair_counts, A, lda,
                                           A32, lda32, s, s1);
    else
        launch_variants<double2, true, 0>(g, L, N, n_if, n_cchunks, q, lists, counts, pairs, pair_counts, A, lda, A32,
                                          lda32, s, s1);
    return hipGetLastError();
}

hipError_t launch_assemble_f32(const char* g, const GeomLayout& L, int N, int n_if, int n_cchunks, int q,
                               const int* const* lists, const int* counts, const int* const* pairs,
                               const int* pair_counts, float2* A, size_t lda, hipStream_t s, hipStream_t s1)
{
    if (q == 8)
        launch_variants<float2, false, 8>(g, L, N, n_if, n_cchunks, q, lists, counts, pairs, pair_counts, A, lda,
                                          nullptr, 0, s, s1);
    else if (q == 10)
        launch_variants<float2, false, 10>(g, L, N, n_if, n_cchunks, q, lists, counts, pairs, pair_counts, A, lda,
                                           nullptr, 0, s, s1);
    else
        launch_variants<float2, false, 0>(g, L, N, n_if, n_cchunks, q, lists, counts, pairs, pair_counts, A, lda,
                                          nullptr, 0, s, s1);
    return hipGetLastError();
}

}  // namespace bemk
