/*
 * bem_oracle.c -- plain, slow, single-threaded FP64 CPU oracle of the
 * collocation BEM of arXiv 2312.12787 (Calderon-ordered Burton-Miller
 * formulation of the 2-D Helmholtz transmission problem).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark to check the HIP path.  It shares no code
 * with the product library.  Everything is written for readability; nothing
 * is blocked, fused or reordered beyond the definitions cited at each step.
 *
 * Steps and where the paper defines them:
 *   geometry        : constant elements, collocation at element centres (Sec. 4, Sec. 7)
 *   Gauss rule      : Gauss-Legendre quadrature (Sec. 7)
 *   kernels         : G = (i/4) H0^(1)(k|x-y|), eq. (fundamental_sol); operators
 *                     S, D, D*, N, eqs. (stmp)-(ddtmp)
 *   self terms      : weak singularity of S and finite part of N (Sec. 7)
 *   block system    : eq. (naive_bie), (calderon_bie1), (calderon_bieb),
 *                     (3dom_conv_bie), (3dom_calderon_bie0), (3dom_calderon_bie)
 *                     and the general recipe closing Sec. 6
 *   right-hand side : u_in + alpha q_in on the host-medium rows (Sec. 3.3, 7)
 *   solve           : dense LU, and GMRES with x0 = 0 (Sec. 3.2, Sec. 7)
 *   far field       : plane-wave asymptotics of the host-medium representation
 *
 * Readings where the paper is silent are stated next to the code and listed in
 * the design notes of the repository.
 */
#include "bem_oracle.h"

#include <complex.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef long double complex lcplx;
typedef double complex dcplx;

static const long double PI_L = 3.141592653589793238462643383279502884L;
static const long double EULER_GAMMA_L = 0.577215664901532860606512090082402431L;

static char g_err[256];
static void set_err(const char *m) { snprintf(g_err, sizeof g_err, "%s", m); }
const char *or_last_error(void) { return g_err; }

/* ------------------------------------------------------------------------- */
/* Gauss-Legendre rule (Sec. 7: Gauss-Legendre quadrature).                   */
/* Newton iteration on the Legendre polynomial P_q evaluated by its three-term */
/* recurrence; weights 2 / ((1 - x^2) P_q'(x)^2).                             */
/* ------------------------------------------------------------------------- */
static void legendre_eval(int q, long double x, long double *pq, long double *dpq)
{
    long double p0 = 1.0L, p1 = x;
    if (q == 0) { *pq = 1.0L; *dpq = 0.0L; return; }
    for (int n = 1; n < q; ++n) {
        long double p2 = ((2.0L * n + 1.0L) * x * p1 - n * p0) / (n + 1.0L);
        p0 = p1;
        p1 = p2;
    }
    *pq = p1;
    *dpq = q * (x * p1 - p0) / (x * x - 1.0L);
}

int or_gauss_legendre(int q, double *xi, double *w)
{
    if (q < 1 || q > 64) { set_err("quadrature order out of range"); return 1; }
    for (int i = 0; i < q; ++i) {
        long double x = cosl(PI_L * (i + 0.75L) / (q + 0.5L));
        for (int it = 0; it < 100; ++it) {
            long double p, dp;
            legendre_eval(q, x, &p, &dp);
            long double dx = p / dp;
            x -= dx;
            if (fabsl(dx) < 1e-19L) break;
        }
        long double p, dp;
        legendre_eval(q, x, &p, &dp);
        /* ascending order of nodes */
        xi[q - 1 - i] = (double)x;
        w[q - 1 - i] = (double)(2.0L / ((1.0L - x * x) * dp * dp));
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Hankel functions H0^(1), H1^(1) for complex z with Im z >= 0.              */
/* Three textbook regimes, all in long double:                                */
/*   |z| <= 8  : ascending series of J0, J1, Y0, Y1 (DLMF 10.2.2, 10.8.1-2);  */
/*   |z| <= 25 : J_n by Miller's backward recurrence normalised with          */
/*               J0 + 2 sum J_2k = 1, Y0 by its Neumann expansion             */
/*               Y0 = (2/pi)(ln(z/2)+gamma) J0 - (4/pi) sum (-1)^k J_2k / k   */
/*               and Y1 = -Y0' differentiated term by term;                   */
/*   |z| > 25  : Hankel's asymptotic expansion (DLMF 10.17.5).                */
/* ------------------------------------------------------------------------- */
static void hankel_series(lcplx z, lcplx *h0, lcplx *h1)
{
    const lcplx q = -z * z / 4.0L; /* (-z^2/4) */
    lcplx lz = clogl(z / 2.0L);
    /* J0 = sum q^k/(k!)^2 ; J1 = (z/2) sum q^k / (k!(k+1)!) */
    lcplx j0 = 0, j1s = 0, y0s = 0, y1s = 0;
    lcplx t0 = 1.0L;  /* q^k/(k!)^2 */
    lcplx t1 = 1.0L;  /* q^k/(k!(k+1)!) */
    long double hk = 0.0L; /* harmonic number H_k */
    for (int k = 0; k < 200; ++k) {
        if (k > 0) {
            t0 *= q / ((long double)k * k);
            t1 *= q / ((long double)k * (k + 1));
            hk += 1.0L / k;
        }
        j0 += t0;
        j1s += t1;
        /* Y0 series part: (2/pi) sum_{k>=1} (-1)^{k+1} H_k (z^2/4)^k/(k!)^2
         *             = -(2/pi) sum_{k>=1} H_k q^k/(k!)^2                    */
        if (k > 0) y0s += -hk * t0;
        /* Y1 series part: psi(k+1) + psi(k+2) = H_k + H_{k+1} - 2 gamma */
        y1s += (hk + (hk + 1.0L / (k + 1)) - 2.0L * EULER_GAMMA_L) * t1;
        if (k > 4 && cabsl(t0) < 1e-22L * cabsl(j0) && cabsl(t1) < 1e-22L * cabsl(j1s)) break;
    }
    lcplx j1 = (z / 2.0L) * j1s;
    lcplx y0 = (2.0L / PI_L) * ((lz + EULER_GAMMA_L) * j0 + y0s);
    /* DLMF 10.8.1 with n = 1 */
    lcplx y1 = -2.0L / (PI_L * z) + (2.0L / PI_L) * lz * j1 - (z / (2.0L * PI_L)) * y1s;
    *h0 = j0 + I * y0;
    *h1 = j1 + I * y1;
}

static void hankel_miller(lcplx z, lcplx *h0, lcplx *h1)
{
    const int M = 2 * ((int)(cabsl(z) / 2.0L) + 30); /* even start index */
    lcplx *J = (lcplx *)calloc((size_t)M + 2, sizeof(lcplx));
    J[M + 1] = 0.0L;
    J[M] = 1e-30L;
    for (int n = M; n >= 1; --n) {
        J[n - 1] = (2.0L * n / z) * J[n] - J[n + 1];
        if (cabsl(J[n - 1]) > 1e300L) { /* rescale to stay finite */
            for (int m = n - 1; m <= M + 1; ++m) J[m] *= 1e-300L;
        }
    }
    lcplx norm = J[0];
    for (int k = 2; k <= M; k += 2) norm += 2.0L * J[k];
    for (int n = 0; n <= M + 1; ++n) J[n] /= norm;
    lcplx lz = clogl(z / 2.0L);
    lcplx s0 = 0, s1 = 0;
    for (int k = 1; 2 * k + 1 <= M + 1; ++k) {
        long double sgn = (k % 2) ? -1.0L : 1.0L;
        s0 += sgn * J[2 * k] / (long double)k;
        s1 += sgn * (J[2 * k - 1] - J[2 * k + 1]) / (long double)k;
    }
    lcplx y0 = (2.0L / PI_L) * (lz + EULER_GAMMA_L) * J[0] - (4.0L / PI_L) * s0;
    /* Y1 = -dY0/dz: J0' = -J1, J_2k' = (J_{2k-1} - J_{2k+1})/2 */
    lcplx y1 = -(2.0L / (PI_L * z)) * J[0] + (2.0L / PI_L) * (lz + EULER_GAMMA_L) * J[1]
               + (2.0L / PI_L) * s1;
    *h0 = J[0] + I * y0;
    *h1 = J[1] + I * y1;
    free(J);
}

static lcplx hankel_asym(int nu, lcplx z)
{
    /* H_nu(z) ~ sqrt(2/(pi z)) e^{i(z - nu pi/2 - pi/4)} sum_k i^k a_k(nu) / z^k,
     * a_k(nu) = prod_{j=1..k} (4 nu^2 - (2j-1)^2) / (k! 8^k)                   */
    const long double mu = 4.0L * nu * nu;
    lcplx sum = 1.0L, term = 1.0L;
    long double prev = 1e300L;
    for (int k = 1; k < 200; ++k) {
        long double odd = 2.0L * k - 1.0L;
        term *= I * (mu - odd * odd) / (k * 8.0L * z);
        long double at = cabsl(term);
        if (at > prev) break; /* the expansion is asymptotic: stop at the smallest term */
        sum += term;
        prev = at;
        if (at < 1e-22L * cabsl(sum)) break;
    }
    lcplx phase = cexpl(I * (z - nu * PI_L / 2.0L - PI_L / 4.0L));
    return csqrtl(2.0L / (PI_L * z)) * phase * sum;
}

static void hankel01_l(lcplx z, lcplx *h0, lcplx *h1)
{
    long double az = cabsl(z);
    if (az <= 8.0L) {
        hankel_series(z, h0, h1);
    } else if (az <= 25.0L) {
        hankel_miller(z, h0, h1);
    } else {
        *h0 = hankel_asym(0, z);
        *h1 = hankel_asym(1, z);
    }
}

int or_hankel01(double zr, double zi, double *out)
{
    if (zi < 0.0 || (zr == 0.0 && zi == 0.0)) { set_err("Hankel argument outside Im z >= 0, z != 0"); return 1; }
    lcplx h0, h1;
    hankel01_l((long double)zr + I * (long double)zi, &h0, &h1);
    out[0] = (double)creall(h0); out[1] = (double)cimagl(h0);
    out[2] = (double)creall(h1); out[3] = (double)cimagl(h1);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Self terms of a flat element at its own midpoint (Sec. 7: the weak          */
/* singularity of S and the hypersingular N are treated analytically).        */
/*   S_ii = int_{-h/2}^{h/2} (i/4) H0(k|s|) ds = (i/(2k)) int_0^{kh/2} H0(t) dt */
/* with the integral taken term by term from the ascending series of J0, Y0,  */
/*   int_0^z (t/2)^{2m} dt         = 2 (z/2)^{2m+1} / (2m+1),                  */
/*   int_0^z ln(t/2) (t/2)^{2m} dt = 2 (z/2)^{2m+1} [ln(z/2)/(2m+1) - 1/(2m+1)^2]. */
/* The finite part of N on its own flat element follows from the identity     */
/*   d2G/dnx dny = k^2 (nx.ny) G - d2G/dtx dty  integrated exactly:           */
/*   N_ii = k^2 S_ii - (i k / 2) H1(k h / 2).                                 */
/* ------------------------------------------------------------------------- */
static lcplx int_h0(lcplx z)
{
    lcplx zh = z / 2.0L, lz = clogl(zh);
    lcplx ij0 = 0, iy0 = 0;
    lcplx p = zh;                 /* (z/2)^{2m+1} */
    long double fact2 = 1.0L;     /* (m!)^2 */
    long double hm = 0.0L;
    for (int m = 0; m < 200; ++m) {
        if (m > 0) {
            p *= zh * zh;
            fact2 *= (long double)m * m;
            hm += 1.0L / m;
        }
        long double sgn = (m % 2) ? -1.0L : 1.0L;
        long double o = 2.0L * m + 1.0L;
        lcplx base = 2.0L * p / fact2;            /* 2 (z/2)^{2m+1}/(m!)^2 */
        lcplx tj = sgn * base / o;
        ij0 += tj;
        /* (2/pi)(ln(t/2)+gamma) J0 part */
        iy0 += (2.0L / PI_L) * sgn * base * ((lz + EULER_GAMMA_L) / o - 1.0L / (o * o));
        /* (2/pi) sum_{m>=1} (-1)^{m+1} H_m (t/2)^{2m}/(m!)^2 part */
        if (m > 0) iy0 += (2.0L / PI_L) * (-sgn) * hm * base / o;
        if (m > 3 && cabsl(tj) < 1e-24L * cabsl(ij0)) break;
    }
    return ij0 + I * iy0;
}

static void self_terms_l(lcplx k, long double h, lcplx *s, lcplx *n)
{
    lcplx z = k * h / 2.0L;
    lcplx sii = (I / (2.0L * k)) * int_h0(z);
    lcplx h0, h1;
    hankel01_l(z, &h0, &h1);
    *s = sii;
    *n = k * k * sii - (I * k / 2.0L) * h1;
}

int or_self_terms(double kr, double ki, double h, double *out)
{
    lcplx s, n;
    self_terms_l((long double)kr + I * (long double)ki, (long double)h, &s, &n);
    out[0] = (double)creall(s); out[1] = (double)cimagl(s);
    out[2] = (double)creall(n); out[3] = (double)cimagl(n);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Problem: geometry, domains, formulation.                                   */
/* ------------------------------------------------------------------------- */
typedef struct {
    double ax, ay, bx, by;  /* end nodes */
    double cx, cy;          /* centre = collocation point */
    double tx, ty;          /* unit tangent */
    double nx, ny;          /* unit normal = left normal (-ty, tx) */
    double h;               /* length */
    int iface;              /* interface index */
} element;

struct or_problem {
    int n_dom, n_if, n_el, quad, form;
    dcplx *k, *eps, *bm_coef;  /* per domain */
    dcplx alpha, beta;
    int *dom_left, *dom_right; /* per interface */
    int *if_offset, *if_count;  /* element ranges per interface */
    element *el;
    double gx[64], gw[64];
    /* row blocks: 2*n_if entries; each: interface, domain, is_bm, row offset */
    int *rb_iface, *rb_dom, *rb_bm, *rb_row0;
    dcplx *rb_scale;   /* standard-type row scaling (beta or 1) */
};

int or_n_elements(const or_problem *p) { return p->n_el; }

void or_problem_free(or_problem *p)
{
    if (!p) return;
    free(p->k); free(p->eps); free(p->bm_coef);
    free(p->dom_left); free(p->dom_right); free(p->if_offset); free(p->if_count);
    free(p->el);
    free(p->rb_iface); free(p->rb_dom); free(p->rb_bm); free(p->rb_row0); free(p->rb_scale);
    free(p);
}

/* sigma_{d m}: +1 if the normal of interface m points out of domain d,
 * -1 if it points into d, 0 if m is not on the boundary of d.               */
static int sigma(const or_problem *p, int d, int m)
{
    if (p->dom_right[m] == d) return 1;
    if (p->dom_left[m] == d) return -1;
    return 0;
}

or_problem *or_problem_new(int n_dom, const double *k, int n_if, const int *n_nodes,
                           const int *closed, const double *xy, const int *dom_left,
                           const int *dom_right, int quad, int form, const double *alpha,
                           const double *beta, const double *bm_coef)
{
    if (n_dom < 2 || n_if < 1 || quad < 1 || quad > 64 || form < 0 || form > 3) {
        set_err("bad problem sizes"); return NULL;
    }
    if (!(k[0] > 0.0) || k[1] != 0.0) { set_err("k0 must be real and positive"); return NULL; }
    or_problem *p = (or_problem *)calloc(1, sizeof *p);
    p->n_dom = n_dom; p->n_if = n_if; p->quad = quad; p->form = form;
    p->k = (dcplx *)malloc(sizeof(dcplx) * n_dom);
    p->eps = (dcplx *)malloc(sizeof(dcplx) * n_dom);
    p->bm_coef = (dcplx *)malloc(sizeof(dcplx) * n_dom);
    for (int d = 0; d < n_dom; ++d) {
        p->k[d] = k[2 * d] + I * k[2 * d + 1];
        if (k[2 * d + 1] < 0.0) { set_err("Im k must be >= 0"); or_problem_free(p); return NULL; }
        /* eps_d = (k_d / k_0)^2 : Sec. 2, k_i = w sqrt(eps_i) with eps_1 = 1 */
        p->eps[d] = (p->k[d] / p->k[0]) * (p->k[d] / p->k[0]);
    }
    /* alpha = -i / k_1 for the host medium (Sec. 3.3) */
    p->alpha = alpha ? (alpha[0] + I * alpha[1]) : (-I / p->k[0]);
    if (beta) p->beta = beta[0] + I * beta[1];
    else p->beta = (form == OR_CALDERON || form == OR_CALDERON_ORIG) ? -p->alpha : 1.0;
    for (int d = 0; d < n_dom; ++d) {
        /* Burton-Miller coefficient alpha / eps_d for domain d (recipe of Sec. 6) */
        p->bm_coef[d] = bm_coef ? (bm_coef[2 * d] + I * bm_coef[2 * d + 1]) : p->alpha / p->eps[d];
    }
    p->dom_left = (int *)malloc(sizeof(int) * n_if);
    p->dom_right = (int *)malloc(sizeof(int) * n_if);
    p->if_offset = (int *)malloc(sizeof(int) * n_if);
    p->if_count = (int *)malloc(sizeof(int) * n_if);
    int total = 0, node0 = 0;
    for (int m = 0; m < n_if; ++m) {
        if (dom_left[m] < 0 || dom_left[m] >= n_dom || dom_right[m] < 0 || dom_right[m] >= n_dom ||
            dom_left[m] == dom_right[m]) {
            set_err("bad domain ids"); or_problem_free(p); return NULL;
        }
        if (dom_left[m] == 0) { set_err("host medium must lie on the side the normal leaves"); or_problem_free(p); return NULL; }
        p->dom_left[m] = dom_left[m];
        p->dom_right[m] = dom_right[m];
        int ne = closed[m] ? n_nodes[m] : n_nodes[m] - 1;
        if (ne < 1 || (closed[m] && n_nodes[m] < 3)) { set_err("too few nodes"); or_problem_free(p); return NULL; }
        p->if_offset[m] = total;
        p->if_count[m] = ne;
        total += ne;
    }
    p->n_el = total;
    p->el = (element *)malloc(sizeof(element) * total);
    for (int m = 0; m < n_if; ++m) {
        int nn = n_nodes[m];
        for (int e = 0; e < p->if_count[m]; ++e) {
            int ia = node0 + e, ib = node0 + ((e + 1) % nn);
            element *E = &p->el[p->if_offset[m] + e];
            E->ax = xy[2 * ia]; E->ay = xy[2 * ia + 1];
            E->bx = xy[2 * ib]; E->by = xy[2 * ib + 1];
            E->cx = 0.5 * (E->ax + E->bx); E->cy = 0.5 * (E->ay + E->by);
            double dx = E->bx - E->ax, dy = E->by - E->ay;
            E->h = sqrt(dx * dx + dy * dy);
            if (!(E->h > 0.0)) { set_err("zero-length element"); or_problem_free(p); return NULL; }
            E->tx = dx / E->h; E->ty = dy / E->h;
            E->nx = -E->ty; E->ny = E->tx;
            E->iface = m;
        }
        node0 += nn;
    }
    or_gauss_legendre(quad, p->gx, p->gw);

    /* Equation blocks: every interface l carries the equation of the domain its
     * normal points into ("left", sigma = -1) and of the domain it leaves
     * ("right", sigma = +1).  Type and placement per formulation:            */
    p->rb_iface = (int *)malloc(sizeof(int) * 2 * n_if);
    p->rb_dom = (int *)malloc(sizeof(int) * 2 * n_if);
    p->rb_bm = (int *)malloc(sizeof(int) * 2 * n_if);
    p->rb_row0 = (int *)malloc(sizeof(int) * 2 * n_if);
    p->rb_scale = (dcplx *)malloc(sizeof(dcplx) * 2 * n_if);
    int nb = 0;
    if (form == OR_CONVENTIONAL) {
        /* eq. (naive_bie) / (3dom_conv_bie): the equations are listed domain by
         * domain as they are written down, host medium first, unscaled.       */
        int row = 0;
        for (int d = 0; d < n_dom; ++d)
            for (int m = 0; m < n_if; ++m) {
                int s = sigma(p, d, m);
                if (!s) continue;
                p->rb_iface[nb] = m; p->rb_dom[nb] = d;
                p->rb_bm[nb] = (d == 0);
                p->rb_scale[nb] = p->beta;
                p->rb_row0[nb] = row;
                row += p->if_count[m];
                ++nb;
            }
    } else {
        /* Calderon forms: standard-type equations in the upper half, scaled by
         * beta; Burton-Miller-type ones in the lower half (end of Sec. 6).    */
        for (int m = 0; m < n_if; ++m) {
            int d = p->dom_left[m];
            p->rb_iface[nb] = m; p->rb_dom[nb] = d; p->rb_bm[nb] = 0;
            p->rb_scale[nb] = p->beta; p->rb_row0[nb] = p->if_offset[m];
            ++nb;
        }
        for (int m = 0; m < n_if; ++m) {
            int d = p->dom_right[m];
            p->rb_iface[nb] = m; p->rb_dom[nb] = d;
            p->rb_bm[nb] = (form == OR_CALDERON_ORIG) ? (d == 0) : 1;
            p->rb_scale[nb] = p->rb_bm[nb] ? 1.0 : p->beta;
            p->rb_row0[nb] = total + p->if_offset[m];
            ++nb;
        }
    }
    return p;
}

int or_elements(const or_problem *p, double *out)
{
    for (int e = 0; e < p->n_el; ++e) {
        const element *E = &p->el[e];
        double v[9] = {E->ax, E->ay, E->bx, E->by, E->cx, E->cy, E->tx, E->ty, E->h};
        memcpy(out + 9 * e, v, sizeof v);
    }
    return 0;
}

int or_normals(const or_problem *p, double *out)
{
    for (int e = 0; e < p->n_el; ++e) { out[2 * e] = p->el[e].nx; out[2 * e + 1] = p->el[e].ny; }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Operator entries between collocation point x_i (centre of element i) and   */
/* element j, for wavenumber k (eqs. (stmp)-(ddtmp), (fundamental_sol)).      */
/* With r = x - y, rh = r/|r|:                                                */
/*   G         = (i/4)   H0(k r)                                              */
/*   dG/dn_y   = (ik/4)  H1(k r) (rh . n_y)                                   */
/*   dG/dn_x   = -(ik/4) H1(k r) (rh . n_x)                                   */
/* S, D, D* of j != i: q-point Gauss-Legendre over element j.  N of j != i:   */
/* the identity d2G/dnx dny = k^2 (nx.ny) G - d2G/dtx dty, exact on a straight */
/* element, turns the finite part into                                        */
/*   N_ij = k^2 (n_i.n_j) S_ij + (ik/4)[H1(k|d_b|)(t_i.d_b)/|d_b|              */
/*                                     - H1(k|d_a|)(t_i.d_a)/|d_a|],          */
/* d_a = x_i - a_j, d_b = x_i - b_j.  Self terms (i = j) are analytic.         */
/* ------------------------------------------------------------------------- */
static void entries(const or_problem *p, dcplx k, int i, int j, dcplx *S, dcplx *D, dcplx *Ds, dcplx *N)
{
    const element *Ei = &p->el[i], *Ej = &p->el[j];
    if (i == j) {
        lcplx s, n;
        self_terms_l((lcplx)k, (long double)Ej->h, &s, &n);
        *S = (dcplx)s; *N = (dcplx)n; *D = 0.0; *Ds = 0.0;
        return;
    }
    dcplx s = 0, d = 0, ds = 0;
    for (int g = 0; g < p->quad; ++g) {
        double sg = 0.5 * Ej->h * p->gx[g];
        double yx = Ej->cx + sg * Ej->tx, yy = Ej->cy + sg * Ej->ty;
        double rx = Ei->cx - yx, ry = Ei->cy - yy;
        double r = sqrt(rx * rx + ry * ry);
        double wgt = 0.5 * Ej->h * p->gw[g];
        lcplx h0, h1;
        hankel01_l((lcplx)(k * r), &h0, &h1);
        dcplx H0 = (dcplx)h0, H1 = (dcplx)h1;
        s += wgt * (I / 4.0) * H0;
        d += wgt * (I * k / 4.0) * H1 * ((rx * Ej->nx + ry * Ej->ny) / r);
        ds += wgt * (-I * k / 4.0) * H1 * ((rx * Ei->nx + ry * Ei->ny) / r);
    }
    double dax = Ei->cx - Ej->ax, day = Ei->cy - Ej->ay;
    double dbx = Ei->cx - Ej->bx, dby = Ei->cy - Ej->by;
    double ra = sqrt(dax * dax + day * day), rb = sqrt(dbx * dbx + dby * dby);
    lcplx h0a, h1a, h0b, h1b;
    hankel01_l((lcplx)(k * ra), &h0a, &h1a);
    hankel01_l((lcplx)(k * rb), &h0b, &h1b);
    dcplx end = (I * k / 4.0) * ((dcplx)h1b * ((Ei->tx * dbx + Ei->ty * dby) / rb)
                                 - (dcplx)h1a * ((Ei->tx * dax + Ei->ty * day) / ra));
    double ninj = Ei->nx * Ej->nx + Ei->ny * Ej->ny;
    *S = s; *D = d; *Ds = ds;
    *N = k * k * ninj * s + end;
}

int or_operator_entries(const or_problem *p, int d, int i, int j, double *out)
{
    if (d < 0 || d >= p->n_dom || i < 0 || j < 0 || i >= p->n_el || j >= p->n_el) { set_err("index"); return 1; }
    dcplx S, D, Ds, N;
    entries(p, p->k[d], i, j, &S, &D, &Ds, &N);
    dcplx v[4] = {S, D, Ds, N};
    memcpy(out, v, sizeof v);
    return 0;
}

/* One row of the system matrix (equation block rb, element i of its interface).
 * Standard equation of domain d at x on interface l (trace of Green's formula,
 * Sec. 3.3 and eq. (3dom_bies)), scaled by s:
 *     s [ 1/2 u_l + sum_m sigma_dm (D_d u_m - eps_d S_d w_m) ]
 * Burton-Miller equation of domain d with coefficient c:
 *     1/2 u_l + sum_m sigma_dm (D_d u_m - eps_d S_d w_m)
 *   + c [ 1/2 eps_d w_l + sum_m sigma_dm (N_d u_m - eps_d D*_d w_m) ]
 * These reproduce eq. (naive_bie) (host medium, sigma = +1, eps = 1, c = alpha;
 * inclusion, sigma = -1) and eq. (3dom_calderon_bie) row by row.            */
static void system_row(const or_problem *p, int rb, int i_local, dcplx *row /* 2N, stride 1 */)
{
    const int N = p->n_el;
    const int l = p->rb_iface[rb], d = p->rb_dom[rb];
    const int i = p->if_offset[l] + i_local;
    const dcplx k = p->k[d], eps = p->eps[d], c = p->bm_coef[d], sc = p->rb_scale[rb];
    const int bm = p->rb_bm[rb];
    for (int col = 0; col < 2 * N; ++col) row[col] = 0.0;
    for (int m = 0; m < p->n_if; ++m) {
        int sg = sigma(p, d, m);
        if (!sg) continue;
        for (int jj = 0; jj < p->if_count[m]; ++jj) {
            int j = p->if_offset[m] + jj;
            dcplx S, D, Ds, Nn;
            entries(p, k, i, j, &S, &D, &Ds, &Nn);
            double delta = (j == i) ? 1.0 : 0.0;
            dcplx au = 0.5 * delta + sg * D;
            dcplx aw = -(double)sg * eps * S;
            if (bm) {
                au += c * (sg * Nn);
                aw += c * (0.5 * eps * delta - sg * eps * Ds);
                row[j] = au;
                row[N + j] = aw;
            } else {
                row[j] = sc * au;
                row[N + j] = sc * aw;
            }
        }
    }
}

static int find_row(const or_problem *p, int row, int *rb, int *il)
{
    for (int b = 0; b < 2 * p->n_if; ++b) {
        int r0 = p->rb_row0[b], cnt = p->if_count[p->rb_iface[b]];
        if (row >= r0 && row < r0 + cnt) { *rb = b; *il = row - r0; return 0; }
    }
    return 1;
}

int or_assemble(const or_problem *p, double *A)
{
    const int n = 2 * p->n_el;
    dcplx *Ac = (dcplx *)A;
    dcplx *row = (dcplx *)malloc(sizeof(dcplx) * n);
    for (int r = 0; r < n; ++r) {
        int rb, il;
        if (find_row(p, r, &rb, &il)) { free(row); set_err("row map"); return 1; }
        system_row(p, rb, il, row);
        for (int c = 0; c < n; ++c) Ac[r + (size_t)c * n] = row[c];
    }
    free(row);
    return 0;
}

int or_assemble_rows(const or_problem *p, int nrows, const int *rows, double *out)
{
    const int n = 2 * p->n_el;
    for (int q = 0; q < nrows; ++q) {
        int rb, il;
        if (rows[q] < 0 || rows[q] >= n || find_row(p, rows[q], &rb, &il)) { set_err("row index"); return 1; }
        system_row(p, rb, il, (dcplx *)out + (size_t)q * n);
    }
    return 0;
}

/* Right-hand side: u_in + c q_in on the rows of the host medium's
 * Burton-Miller equation (eq. (calderon_bieb)), 0 elsewhere; plane wave
 * u_in = exp(i k0 d.x), q_in = du_in/dn = i k0 (d.n) u_in (Sec. 7).        */
int or_rhs(const or_problem *p, int nang, const double *angles, double *B)
{
    const int n = 2 * p->n_el;
    dcplx *Bc = (dcplx *)B;
    const double k0 = creal(p->k[0]);
    for (int a = 0; a < nang; ++a) {
        double dx = cos(angles[a]), dy = sin(angles[a]);
        for (int r = 0; r < n; ++r) Bc[r + (size_t)a * n] = 0.0;
        for (int rb = 0; rb < 2 * p->n_if; ++rb) {
            if (p->rb_dom[rb] != 0) continue;
            int l = p->rb_iface[rb];
            dcplx c = p->rb_bm[rb] ? p->bm_coef[0] : 0.0;
            dcplx sc = p->rb_bm[rb] ? 1.0 : p->rb_scale[rb];
            for (int e = 0; e < p->if_count[l]; ++e) {
                const element *E = &p->el[p->if_offset[l] + e];
                dcplx uin = cexp(I * k0 * (dx * E->cx + dy * E->cy));
                dcplx qin = I * k0 * (dx * E->nx + dy * E->ny) * uin;
                Bc[p->rb_row0[rb] + e + (size_t)a * n] = sc * (uin + c * qin);
            }
        }
    }
    return 0;
}

void or_matvec(int n, const double *A, const double *x, double *y)
{
    const dcplx *Ac = (const dcplx *)A, *xc = (const dcplx *)x;
    dcplx *yc = (dcplx *)y;
    for (int r = 0; r < n; ++r) {
        dcplx s = 0.0;
        for (int c = 0; c < n; ++c) s += Ac[r + (size_t)c * n] * xc[c];
        yc[r] = s;
    }
}

int or_lu_solve(int n, double *A, int nrhs, double *B)
{
    dcplx *a = (dcplx *)A, *b = (dcplx *)B;
#define AA(r, c) a[(r) + (size_t)(c) * n]
    for (int col = 0; col < n; ++col) {
        int piv = col;
        double best = cabs(AA(col, col));
        for (int r = col + 1; r < n; ++r)
            if (cabs(AA(r, col)) > best) { best = cabs(AA(r, col)); piv = r; }
        if (best == 0.0) return 1;
        if (piv != col) {
            for (int c = 0; c < n; ++c) { dcplx t = AA(col, c); AA(col, c) = AA(piv, c); AA(piv, c) = t; }
            for (int c = 0; c < nrhs; ++c) {
                dcplx t = b[col + (size_t)c * n]; b[col + (size_t)c * n] = b[piv + (size_t)c * n]; b[piv + (size_t)c * n] = t;
            }
        }
        for (int r = col + 1; r < n; ++r) {
            dcplx f = AA(r, col) / AA(col, col);
            AA(r, col) = f;
            for (int c = col + 1; c < n; ++c) AA(r, c) -= f * AA(col, c);
            for (int c = 0; c < nrhs; ++c) b[r + (size_t)c * n] -= f * b[col + (size_t)c * n];
        }
    }
    for (int c = 0; c < nrhs; ++c) {
        dcplx *x = b + (size_t)c * n;
        for (int r = n - 1; r >= 0; --r) {
            dcplx s = x[r];
            for (int q = r + 1; q < n; ++q) s -= AA(r, q) * x[q];
            x[r] = s / AA(r, r);
        }
    }
#undef AA
    return 0;
}

static double vnorm(int n, const dcplx *v)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += creal(v[i]) * creal(v[i]) + cimag(v[i]) * cimag(v[i]);
    return sqrt(s);
}

/* GMRES(m) (Saad and Schultz) with x0 = 0 (Sec. 3.2: the Krylov space of A
 * spanned from b).  Arnoldi by modified Gram-Schmidt; the small least-squares
 * problem by Givens rotations.                                               */
int or_gmres(int n, const double *A, const double *b, int m, double tol, int max_it,
             double *x, int *iters, double *relres)
{
    const dcplx *bc = (const dcplx *)b;
    dcplx *xc = (dcplx *)x;
    dcplx *V = (dcplx *)calloc((size_t)n * (m + 1), sizeof(dcplx));
    dcplx *H = (dcplx *)calloc((size_t)(m + 1) * m, sizeof(dcplx));
    dcplx *cs = (dcplx *)calloc(m, sizeof(dcplx)), *sn = (dcplx *)calloc(m, sizeof(dcplx));
    dcplx *g = (dcplx *)calloc(m + 1, sizeof(dcplx)), *y = (dcplx *)calloc(m, sizeof(dcplx));
    dcplx *r = (dcplx *)calloc(n, sizeof(dcplx)), *w = (dcplx *)calloc(n, sizeof(dcplx));
    for (int i = 0; i < n; ++i) xc[i] = 0.0;
    const double bnorm = vnorm(n, bc);
    int it = 0, converged = 0;
    double rel = 1.0;
    if (bnorm == 0.0) { converged = 1; rel = 0.0; }
#define HH(i, j) H[(i) + (size_t)(j) * (m + 1)]
    while (!converged && it < max_it) {
        /* r = b - A x */
        or_matvec(n, A, x, (double *)w);
        if (it > 0) ++it; /* the explicit residual of a restart costs one product */
        for (int i = 0; i < n; ++i) r[i] = bc[i] - w[i];
        double beta = vnorm(n, r);
        rel = beta / bnorm;
        if (rel <= tol) { converged = 1; break; }
        for (int i = 0; i < n; ++i) V[i] = r[i] / beta;
        for (int i = 0; i <= m; ++i) g[i] = 0.0;
        g[0] = beta;
        int j;
        for (j = 0; j < m && it < max_it; ++j) {
            or_matvec(n, A, (const double *)(V + (size_t)j * n), (double *)w);
            ++it;
            for (int i = 0; i <= j; ++i) {
                dcplx h = 0.0;
                for (int q = 0; q < n; ++q) h += conj(V[q + (size_t)i * n]) * w[q];
                HH(i, j) = h;
                for (int q = 0; q < n; ++q) w[q] -= h * V[q + (size_t)i * n];
            }
            double hn = vnorm(n, w);
            HH(j + 1, j) = hn;
            if (hn > 0.0)
                for (int q = 0; q < n; ++q) V[q + (size_t)(j + 1) * n] = w[q] / hn;
            for (int i = 0; i < j; ++i) { /* apply earlier rotations */
                dcplx t = cs[i] * HH(i, j) + sn[i] * HH(i + 1, j);
                HH(i + 1, j) = -conj(sn[i]) * HH(i, j) + conj(cs[i]) * HH(i + 1, j);
                HH(i, j) = t;
            }
            /* new rotation zeroing H(j+1, j) */
            dcplx a = HH(j, j), bb = HH(j + 1, j);
            double den = sqrt(creal(a * conj(a)) + creal(bb * conj(bb)));
            if (den == 0.0) { cs[j] = 1.0; sn[j] = 0.0; }
            else if (cabs(a) == 0.0) { cs[j] = 0.0; sn[j] = conj(bb) / cabs(bb); }
            else { cs[j] = cabs(a) / den; sn[j] = (a / cabs(a)) * conj(bb) / den; }
            HH(j, j) = cs[j] * a + sn[j] * bb;
            HH(j + 1, j) = 0.0;
            g[j + 1] = -conj(sn[j]) * g[j];
            g[j] = cs[j] * g[j];
            rel = cabs(g[j + 1]) / bnorm;
            if (rel <= tol || hn == 0.0) { ++j; break; }
        }
        /* solve the triangular system and update x */
        for (int i = j - 1; i >= 0; --i) {
            dcplx s = g[i];
            for (int q = i + 1; q < j; ++q) s -= HH(i, q) * y[q];
            y[i] = s / HH(i, i);
        }
        for (int i = 0; i < j; ++i)
            for (int q = 0; q < n; ++q) xc[q] += y[i] * V[q + (size_t)i * n];
        /* true residual decides convergence */
        or_matvec(n, A, x, (double *)w);
        for (int i = 0; i < n; ++i) r[i] = bc[i] - w[i];
        rel = vnorm(n, r) / bnorm;
        if (rel <= tol) converged = 1;
        else if (it >= max_it) break;
        else --it; /* the next restart's residual product is this one */
    }
#undef HH
    *iters = it;
    *relres = rel;
    free(V); free(H); free(cs); free(sn); free(g); free(y); free(r); free(w);
    return converged ? 0 : 1;
}

/* Far field of the scattered field in the host medium.  The host-medium
 * representation u = u_in + sum_m sigma_0m (S_0 w_m - D_0 u_m) (eps_0 = 1)
 * with the large-|x| form of G gives u_sc ~ e^{ik0|x|}/sqrt|x| F(xh),
 *   F(xh) = e^{i pi/4}/sqrt(8 pi k0) sum_j sigma_0j [w_j + i k0 (xh.n_j) u_j]
 *           h_j e^{-i k0 xh.c_j} sinc(k0 h_j xh.t_j / 2)
 * (the element integral of e^{-i k0 xh.y} done exactly; sinc(a) = sin a / a). */
int or_farfield(const or_problem *p, int nrhs, const double *X, int ndir, const double *dirs,
                double *F)
{
    const int N = p->n_el, n = 2 * N;
    const dcplx *Xc = (const dcplx *)X;
    dcplx *Fc = (dcplx *)F;
    const double k0 = creal(p->k[0]);
    const dcplx pref = cexp(I * (double)PI_L / 4.0) / sqrt(8.0 * (double)PI_L * k0);
    for (int r = 0; r < nrhs; ++r)
        for (int q = 0; q < ndir; ++q) {
            double xh = cos(dirs[q]), yh = sin(dirs[q]);
            dcplx s = 0.0;
            for (int m = 0; m < p->n_if; ++m) {
                int sg = sigma(p, 0, m);
                if (!sg) continue;
                for (int e = 0; e < p->if_count[m]; ++e) {
                    int j = p->if_offset[m] + e;
                    const element *E = &p->el[j];
                    dcplx u = Xc[j + (size_t)r * n], w = Xc[N + j + (size_t)r * n];
                    double a = 0.5 * k0 * E->h * (xh * E->tx + yh * E->ty);
                    double sinc = (a == 0.0) ? 1.0 : sin(a) / a;
                    s += sg * (w + I * k0 * (xh * E->nx + yh * E->ny) * u) * E->h
                         * cexp(-I * k0 * (xh * E->cx + yh * E->cy)) * sinc;
                }
            }
            Fc[q + (size_t)r * ndir] = pref * s;
        }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Near field (Sec. 7.1: the total field at field points).  A point x in     */
/* domain d takes Green's representation formula of that domain with the     */
/* boundary data (u_j, w_j = (1/eps) du/dn) of the solution:                  */
/*   u(x) = [d = host] u_in(x)                                               */
/*        + sum_m sigma_dm sum_{j in m} ( eps_d int_j G_d(x-y) ds_y w_j       */
/*                                        - int_j dG_d/dn_y(x-y) ds_y u_j ),  */
/* sigma_dm = +1 where the normal leaves d (it is then d's outward normal).   */
/* Element integrals: adaptive Gauss-Legendre bisection (10 points on each    */
/* half against 10 on the whole, until they agree to 1e-13 relative or to an  */
/* absolute floor of 1e-16 of the element's scale), which resolves the peaked */
/* integrands of points close to the boundary.                                */
/* ------------------------------------------------------------------------- */
static double nf_gx[10], nf_gw[10];
static int nf_rule_ready = 0;

/* The integrands in the element's own coordinates: xt = (x - a).t, xn = (x - a).n,
 * so that r^2 = (xt - s)^2 + xn^2 keeps full relative accuracy for points very
 * close to the element (forming y(s) and x - y in global coordinates would
 * lose it to cancellation). */
static void nf_rule(double s0, double s1, dcplx k, double xt, double xn, dcplx *S, dcplx *D)
{
    dcplx s = 0, d = 0;
    const double half = 0.5 * (s1 - s0), mid = 0.5 * (s0 + s1);
    for (int g = 0; g < 10; ++g) {
        const double sg = mid + half * nf_gx[g];  /* arclength from node a */
        const double u = xt - sg;
        const double r = sqrt(u * u + xn * xn);
        lcplx h0, h1;
        hankel01_l((lcplx)(k * r), &h0, &h1);
        const double wgt = half * nf_gw[g];
        s += wgt * (I / 4.0) * (dcplx)h0;
        d += wgt * (I * k / 4.0) * (dcplx)h1 * (xn / r);
    }
    *S = s;
    *D = d;
}

static void nf_adapt(double s0, double s1, dcplx k, double xt, double xn, dcplx Sw, dcplx Dw, double floor_,
                     int depth, dcplx *S, dcplx *D)
{
    const double m = 0.5 * (s0 + s1);
    dcplx S1, D1, S2, D2;
    nf_rule(s0, m, k, xt, xn, &S1, &D1);
    nf_rule(m, s1, k, xt, xn, &S2, &D2);
    const dcplx Sh = S1 + S2, Dh = D1 + D2;
    const double diff = cabs(Sh - Sw) + cabs(Dh - Dw);
    const double size = cabs(Sh) + cabs(Dh);
    if (diff <= 1e-13 * size || diff <= floor_ || depth >= 40) {
        *S = Sh;
        *D = Dh;
        return;
    }
    dcplx Sa, Da, Sb, Db;
    nf_adapt(s0, m, k, xt, xn, S1, D1, floor_, depth + 1, &Sa, &Da);
    nf_adapt(m, s1, k, xt, xn, S2, D2, floor_, depth + 1, &Sb, &Db);
    *S = Sa + Sb;
    *D = Da + Db;
}

int or_nearfield(const or_problem *p, int nrhs, const double *X, const double *angles, int npts,
                 const double *xy, const int *dom, double *U)
{
    const int N = p->n_el, n = 2 * N;
    const dcplx *Xc = (const dcplx *)X;
    dcplx *Uc = (dcplx *)U;
    if (!nf_rule_ready) {
        or_gauss_legendre(10, nf_gx, nf_gw);
        nf_rule_ready = 1;
    }
    for (int pt = 0; pt < npts; ++pt) {
        const int d = dom[pt];
        if (d < 0 || d >= p->n_dom) { set_err("domain of a field point out of range"); return 1; }
        const double x = xy[2 * pt], y = xy[2 * pt + 1];
        const dcplx k = p->k[d], eps = p->eps[d];
        for (int r = 0; r < nrhs; ++r) Uc[pt + (size_t)r * npts] = 0.0;
        for (int m = 0; m < p->n_if; ++m) {
            const int sg = sigma(p, d, m);
            if (!sg) continue;
            for (int e = 0; e < p->if_count[m]; ++e) {
                const int j = p->if_offset[m] + e;
                const element *E = &p->el[j];
                const double xt = (x - E->ax) * E->tx + (y - E->ay) * E->ty;
                const double xn = (x - E->ax) * E->nx + (y - E->ay) * E->ny;
                dcplx Sw, Dw, S, D;
                nf_rule(0.0, E->h, k, xt, xn, &Sw, &Dw);
                /* absolute floor: 1e-16 of a bound on the element's integrals */
                const double floor_ = 1e-16 * (cabs(Sw) + cabs(Dw) + E->h * cabs(k) + 1.0);
                nf_adapt(0.0, E->h, k, xt, xn, Sw, Dw, floor_, 0, &S, &D);
                for (int r = 0; r < nrhs; ++r) {
                    const dcplx u = Xc[j + (size_t)r * n], w = Xc[N + j + (size_t)r * n];
                    Uc[pt + (size_t)r * npts] += sg * (eps * S * w - D * u);
                }
            }
        }
        if (d == 0 && angles)
            for (int r = 0; r < nrhs; ++r) {
                const double k0 = creal(p->k[0]);
                Uc[pt + (size_t)r * npts] += cexp(I * k0 * (cos(angles[r]) * x + sin(angles[r]) * y));
            }
    }
    return 0;
}
