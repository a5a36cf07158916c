// linalg.hip -- right-hand sides and the batched GMRES(m) building blocks (Sec. 3.2: GMRES on A itself, x0 = 0),
// plus the far-field output step.
//
// Layouts: matrices column-major; a block of vectors is column-major with one
// column per right-hand side.  The Krylov basis of all right-hand sides is
// V[(i * nr + r) * ldv + q] (basis vector i of right-hand side r, row q).
// All reductions run in a fixed order, so repeated runs are bitwise equal.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#include "bem.h"
#include "internal.h"
#include "krylov_dev.h"
#include "launch.h"

namespace bemk {

namespace {

constexpr int BS = 256;        // threads per block

template <class T>
__device__ __forceinline__ const T* tab(const char* g, size_t off) { return reinterpret_cast<const T*>(g + off); }

// Krylov basis entries: complex128, or complex64 (the FP32-product solves)
// widened on load and rounded on store; all arithmetic stays FP64.
__device__ __forceinline__ double2 ld2(const double2* p) { return *p; }
__device__ __forceinline__ double2 ld2(const float2* p)
{
    const float2 f = *p;
    return make_double2(f.x, f.y);
}
__device__ __forceinline__ void st2(double2* p, double2 v) { *p = v; }
__device__ __forceinline__ void st2(float2* p, double2 v) { *p = make_float2((float)v.x, (float)v.y); }

using dev::STOPPING;
using dev::wave_sum;

// Sum NV values over the 256 threads of a block; result valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* lds /* [4][NV] */)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) lds[wave * NV + k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] = lds[k] + lds[NV + k] + lds[2 * NV + k] + lds[3 * NV + k];
}

// ---------------------------------------------------------------------------
// Plane-wave right-hand sides (Sec. 7: u_in = exp(i k0 d.x); eq. (calderon_bieb):
// u_in + alpha q_in on the host medium's Burton-Miller rows, 0 elsewhere).
// ---------------------------------------------------------------------------
__global__ void k_rhs(const char* __restrict__ g, GeomLayout L, int N, AngleChunk angles, int nang,
                      double2* __restrict__ B, size_t ldb)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (e >= N || r >= nang) return;
    const ElemRec E = tab<ElemRec>(g, L.elem)[e];
    const IfacePlan P = tab<IfacePlan>(g, L.iface)[tab<int>(g, L.elif)[e]];
    const DomConst D0 = tab<DomConst>(g, L.dom)[0];
    const double k0 = D0.k[0];
    double sd, cd_;
    sincos(angles.v[r], &sd, &cd_);
    double sp, cp;
    sincos(k0 * (cd_ * E.cx + sd * E.cy), &sp, &cp);  // u_in = cp + i sp
    const double dn = k0 * (cd_ * E.nx + sd * E.ny);   // q_in = i dn u_in
    const double qr = -dn * sp, qi = dn * cp;
    double2* col = B + (size_t)r * ldb;
    col[P.row_l + (e - P.off)] = make_double2(0.0, 0.0);  // dom_left is never the host medium
    double2 v = make_double2(0.0, 0.0);
    if (P.dr == 0) {
        if (P.bm_r) {
            v.x = cp + D0.c[0] * qr - D0.c[1] * qi;
            v.y = sp + D0.c[0] * qi + D0.c[1] * qr;
        } else {
            v.x = D0.beta[0] * cp - D0.beta[1] * sp;
            v.y = D0.beta[0] * sp + D0.beta[1] * cp;
        }
    }
    col[P.row_r + (e - P.off)] = v;
}

// ---------------------------------------------------------------------------
// GMRES pieces.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BS) void k_col_norm_partial(const double2* __restrict__ X, size_t ldx, int n,
                                                         double* __restrict__ partial)
{
    __shared__ double lds[4];
    const int r = blockIdx.y;
    double acc[1] = {0.0};
    for (int q = blockIdx.x * BS + threadIdx.x; q < n; q += gridDim.x * BS) {
        const double2 v = X[(size_t)r * ldx + q];
        acc[0] = fma(v.x, v.x, fma(v.y, v.y, acc[0]));
    }
    block_sum<1>(acc, lds);
    if (threadIdx.x == 0) partial[r * gridDim.x + blockIdx.x] = acc[0];
}

__global__ void k_col_norm_finish(const double* __restrict__ partial, int nblk, int nr, double* __restrict__ out)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += partial[r * nblk + b];
    out[r] = sqrt(s);
}









// y = H(0:k, 0:k)^{-1} g(0:k), column-oriented back substitution: one wave per
// right-hand side, g in LDS; step i divides by H(i, i) and removes column i
// from the rows above it (lanes over rows).
__global__ __launch_bounds__(64) void k_backsolve_wave(int nr, int m, const double2* __restrict__ H,
                                                       const double2* __restrict__ gvec,
                                                       const int* __restrict__ kdim, double2* __restrict__ y)
{
    extern __shared__ double2 g[];  // m entries
    __shared__ double2 yi_s;
    const int r = blockIdx.x;
    const int k = kdim[r];
    const int lane = threadIdx.x;
    if (k == 0) return;
    const double2* Hr = H + (size_t)r * (m + 1) * m;
    for (int i = lane; i < k; i += 64) g[i] = gvec[(size_t)r * (m + 1) + i];
    __syncthreads();
    for (int i = k - 1; i >= 0; --i) {
        if (lane == 0) {
            const double2 d = Hr[i + (size_t)i * (m + 1)];
            const double den = d.x * d.x + d.y * d.y;
            const double2 v = g[i];
            const double2 yi = den > 0.0 ? make_double2((v.x * d.x + v.y * d.y) / den, (v.y * d.x - v.x * d.y) / den)
                                         : make_double2(0.0, 0.0);
            yi_s = yi;
            y[(size_t)r * (m + 1) + i] = yi;
        }
        __syncthreads();
        const double2 yi = yi_s;
        for (int p = lane; p < i; p += 64) {
            const double2 h = Hr[p + (size_t)i * (m + 1)];
            double2 v = g[p];
            v.x -= h.x * yi.x - h.y * yi.y;
            v.y -= h.x * yi.y + h.y * yi.x;
            g[p] = v;
        }
        __syncthreads();
    }
}


// ---------------------------------------------------------------------------
// Arnoldi step with delayed re-orthogonalisation and device-side control.
// At step j the basis v_0..v_{j-1} is final, the candidate vt = V_j has had one
// Gram-Schmidt pass and unit norm, and (j < m) wt = A vt.  One projection pass
// gives s = V_{<j}^H vt, alpha = |vt|^2, t = V_{<j}^H wt, tau = vt^H wt; with
// V_{<j} orthonormal the rest is exact algebra:
//   gamma = sqrt(alpha - |s|^2),  v_j = (vt - V_{<j} s) / gamma,
//   column j-1 of the Hessenberg matrix gains beta s, H[j, j-1] = beta gamma
//   (beta = |w| of step j-1), which completes it: Givens rotation, residual
//   estimate and stopping decision for Krylov dimension j;
//   z = H[0:j+1, 0:j] s,  c = (tau - s^H t) / gamma,
//   column j: H[i, j] = (t_i - z_i) / gamma (i < j),  H[j, j] = (c - z_j) / gamma,
//   w = (wt - V_{<j} t - v_j c) / gamma,  beta = |w|,  V_{j+1} = w / beta.
// Two passes over the basis per step (projection, update) instead of the four
// of classical Gram-Schmidt with a second pass; the product of the step at
// which a column stops is not used.  Reductions run in a fixed order.
// ---------------------------------------------------------------------------

// Partial projections of the candidate (and of wt when HASW) on V_0..V_j for a
// batch of BATCH basis vectors, one right-hand side r and one chunk of
// rpt * BS rows: partP/partQ[(r * ns + chunk) * jc + i].  One-dimensional
// grid of rcp * batches blocks, block b taking (right-hand side, chunk) pair
// b % rcp and batch b / rcp, with rcp = nr * ns rounded up to a multiple of 8:
// workgroups go to the eight XCDs in turn, so every batch of one (right-hand
// side, chunk) runs on the same XCD and reads its candidate and wt rows from
// that XCD's L2 after the first batch brought them in (ids >= nr * ns of a
// padded row exit at once; measured on gfx950 for kite4096 with 16
// right-hand sides: 534.9 against 530.7 solves/s with the batches of one pair
// on consecutive ids).  Adding the product's split partial sums here instead
// of in its own reduction pass was slower (525.9), every batch re-reading them.
template <int BATCH, bool HASW, class TV>
__device__ __forceinline__ void dc_dots(int bid, const TV* __restrict__ V, size_t ldv, int nr, int jc,
                                        const double2* __restrict__ W, size_t ldw, int n, int rpt, int ns, int rcp,
                                        double2* __restrict__ partP, double2* __restrict__ partQ,
                                        const int* __restrict__ active)
{
    constexpr int NV = (HASW ? 4 : 2) * BATCH;
    __shared__ double lds[4 * NV];
    const int rc = (int)((unsigned)bid % (unsigned)rcp);
    if (rc >= nr * ns) return;
    const int r = rc % nr, chunk = rc / nr;
    const int i0 = (int)((unsigned)bid / (unsigned)rcp) * BATCH;
    if (!active[r]) return;
    double acc[NV];
#pragma unroll
    for (int b = 0; b < NV; ++b) acc[b] = 0.0;
    const size_t vstride = (size_t)nr * ldv;
    const TV* vb = V + ((size_t)i0 * nr + r) * ldv;
    const TV* vt = V + ((size_t)(jc - 1) * nr + r) * ldv;
    const double2* wr = HASW ? W + (size_t)r * ldw : nullptr;
    const int nb = min(BATCH, jc - i0);
    const int q0 = chunk * rpt * BS + threadIdx.x;
    const int q1 = min(n, (chunk + 1) * rpt * BS);
    // one row's contribution to every accumulator, in the same order for
    // both loops below
    auto row = [&](const double2 a, const double2 w, const double2* v, int cnt) {
#pragma unroll
        for (int b = 0; b < BATCH; ++b) {
            if (b < cnt) {
                acc[2 * b] = fma(v[b].x, a.x, fma(v[b].y, a.y, acc[2 * b]));
                acc[2 * b + 1] = fma(v[b].x, a.y, fma(-v[b].y, a.x, acc[2 * b + 1]));
                if (HASW) {
                    acc[2 * BATCH + 2 * b] = fma(v[b].x, w.x, fma(v[b].y, w.y, acc[2 * BATCH + 2 * b]));
                    acc[2 * BATCH + 2 * b + 1] = fma(v[b].x, w.y, fma(-v[b].y, w.x, acc[2 * BATCH + 2 * b + 1]));
                }
            }
        }
    };
    if (nb == BATCH) {
        // full batch: every load of two rows is issued before the first use
        // (the per-vector guard of the partial batch below makes the compiler
        // wait for each load in turn); the loads share one 32-bit byte offset
        // from wave-uniform bases, so they take no per-load address registers
        const char* bv[BATCH];
#pragma unroll
        for (int b = 0; b < BATCH; ++b) bv[b] = reinterpret_cast<const char*>(vb + b * vstride);
        const char* bt = reinterpret_cast<const char*>(vt);
        const char* bw = reinterpret_cast<const char*>(wr);
        auto at = [](const char* base, unsigned off) { return ld2(reinterpret_cast<const TV*>(base + off)); };
        auto aw = [](const char* base, unsigned off) { return *reinterpret_cast<const double2*>(base + off); };
        int q = q0;
        for (; q + BS < q1; q += 2 * BS) {
            double2 a[2], w[2] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0)}, v[2][BATCH];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const unsigned qo = (unsigned)(q + u * BS);
                a[u] = at(bt, qo * (unsigned)sizeof(TV));
                if (HASW) w[u] = aw(bw, qo * (unsigned)sizeof(double2));
#pragma unroll
                for (int b = 0; b < BATCH; ++b) v[u][b] = at(bv[b], qo * (unsigned)sizeof(TV));
            }
            row(a[0], w[0], v[0], BATCH);
            row(a[1], w[1], v[1], BATCH);
        }
        if (q < q1) {
            double2 v[BATCH];
            const unsigned qo = (unsigned)q;
            const double2 a = at(bt, qo * (unsigned)sizeof(TV));
            const double2 w = HASW ? aw(bw, qo * (unsigned)sizeof(double2)) : make_double2(0.0, 0.0);
#pragma unroll
            for (int b = 0; b < BATCH; ++b) v[b] = at(bv[b], qo * (unsigned)sizeof(TV));
            row(a, w, v, BATCH);
        }
    } else {
        for (int q = q0; q < q1; q += BS) {
            double2 v[BATCH];
            const double2 a = ld2(vt + q);
            const double2 w = HASW ? wr[q] : make_double2(0.0, 0.0);
#pragma unroll
            for (int b = 0; b < BATCH; ++b)
                if (b < nb) v[b] = ld2(vb + b * vstride + q);
            row(a, w, v, nb);
        }
    }
    // block sums in block_sum's order (each wave's DPP sum, then waves 0..3),
    // finished by one thread per (real, imaginary) pair so that no thread
    // holds all of them
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = wave_sum(acc[k]);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) lds[wave * NV + k] = acc[k];
    __syncthreads();
    const int t = threadIdx.x;
    if (t < NV / 2) {
        const int k = 2 * t;
        const double re = lds[k] + lds[NV + k] + lds[2 * NV + k] + lds[3 * NV + k];
        const double im = lds[k + 1] + lds[NV + k + 1] + lds[2 * NV + k + 1] + lds[3 * NV + k + 1];
        const int b = t < BATCH ? t : t - BATCH;  // pairs BATCH.. are the wt projections
        if (b < nb) {
            const size_t o = ((size_t)r * ns + chunk) * jc + i0 + b;
            if (t < BATCH)
                partP[o] = make_double2(re, im);
            else
                partQ[o] = make_double2(re, im);
        }
    }
}

__device__ __forceinline__ double2 cmul2(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// The small work of step j for one right-hand side (one block): sum the
// projection partials into S = [s, alpha] and T = [t, tau], complete column
// j-1 (Givens, residual, decision) and form column j.  Hraw holds the
// Hessenberg matrix as produced, H its rotated (triangular) form for the
// back-solve.  It runs in the update launch, beside the blocks that apply
// the update (which form the same S, T, gamma and c themselves).
constexpr int DC_STEP_BS = 256;  // threads of a step block

// three sums over the workgroup with one barrier, each in a fixed order: the
// wave's DPP sum, then waves 0..3
__device__ __forceinline__ void block_sum4x3(double& a, double& b, double& c, double* red)
{
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    if ((threadIdx.x & 63) == 0) {
        const int w = threadIdx.x >> 6;
        red[w] = a;
        red[4 + w] = b;
        red[8 + w] = c;
    }
    __syncthreads();
    a = ((red[0] + red[1]) + red[2]) + red[3];
    b = ((red[4] + red[5]) + red[6]) + red[7];
    c = ((red[8] + red[9]) + red[10]) + red[11];
}

// LDS of the step and update blocks (double2 units): five arrays of m + 1
// entries, the wave partials zp[4][64], then reduction slots and a flag.
__host__ __device__ constexpr size_t arn_lds_elems(int m) { return 5 * ((size_t)m + 1) + 4 * 64 + 16; }
static_assert(arn_lds_elems(BEM_MAX_RESTART) * sizeof(double2) <= 160 * 1024,
              "a step block of the longest restart fits the 160 KiB of LDS a gfx950 workgroup can hold");

// A column that stops at step j of a cycle (convergence, spent budget, end of
// the Krylov space) is marked STOPPING in `active` while the update blocks of
// the same launch may still read it (they update columns marked 1 or
// STOPPING; the update of a stopping column is never used), and the
// normalisation that follows clears the mark; at the last step of a cycle it
// is cleared at once.

__device__ __forceinline__ void dc_step(int r, int nr, int j, int m, int ns, const double2* __restrict__ partP,
                                        const double2* __restrict__ partQ, double2* __restrict__ Hraw,
                                        double2* __restrict__ H, double2* __restrict__ cs, double2* __restrict__ sn,
                                        double2* __restrict__ gvec, const double* __restrict__ hnorm,
                                        const double* __restrict__ thr, int maxit, int* __restrict__ iters,
                                        int* __restrict__ kdim, int* __restrict__ active,
                                        int* __restrict__ flags_out, double2* __restrict__ lds)
{
    // S, T and the column being completed stay in LDS for the whole step; the
    // inputs of earlier steps (column j - 1 as produced, the rotations, the
    // rotated right-hand side) are loaded first, alongside the partial sums
    const size_t L = (size_t)m + 1;
    double2* col = lds;
    double2* lc = lds + L;
    double2* ls = lds + 2 * L;
    double2* Sl = lds + 3 * L;
    double2* Tl = lds + 4 * L;
    double2(*zp)[64] = reinterpret_cast<double2(*)[64]>(lds + 5 * L);
    double* red = reinterpret_cast<double*>(lds + 5 * L + 4 * 64);
    int* still_p = reinterpret_cast<int*>(red + 16);
    int& still_s = *still_p;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int stop_mark = j == m ? 0 : STOPPING;
    if (!active[r]) {
        if (flags_out && tid == 0) flags_out[r] = 0;
        return;
    }
    const int jc = j + 1;
    const bool hasw = partQ != nullptr;
    double2* Hc = Hraw + (size_t)r * (m + 1) * m + (size_t)(j >= 1 ? j - 1 : 0) * (m + 1);
    if (j >= 1) {
        for (int i = tid; i < j; i += DC_STEP_BS) col[i] = Hc[i];
        for (int i = tid; i < j - 1; i += DC_STEP_BS) {
            lc[i] = cs[(size_t)r * m + i];
            ls[i] = sn[(size_t)r * m + i];
        }
    }
    for (int i = tid; i < jc; i += DC_STEP_BS) {
        double pr = 0.0, pi = 0.0, qr = 0.0, qi = 0.0;
#pragma unroll 8
        for (int b = 0; b < ns; ++b) {
            const size_t o = ((size_t)r * ns + b) * jc + i;
            const double2 p = partP[o];
            pr += p.x;
            pi += p.y;
            if (hasw) {
                const double2 t = partQ[o];
                qr += t.x;
                qi += t.y;
            }
        }
        Sl[i] = make_double2(pr, pi);
        if (hasw) Tl[i] = make_double2(qr, qi);
    }
    __syncthreads();
    const double beta = j >= 1 ? hnorm[r] : 1.0;
    const bool brk = !(beta > 0.0);  // previous step ended the Krylov space
    double ss = 0.0, str = 0.0, sti = 0.0;
    for (int i = tid; i < j; i += DC_STEP_BS) {
        const double2 a = brk ? make_double2(0.0, 0.0) : Sl[i];
        ss = fma(a.x, a.x, fma(a.y, a.y, ss));
        if (hasw) {
            const double2 t = Tl[i];
            str = fma(a.x, t.x, fma(a.y, t.y, str));
            sti = fma(a.x, t.y, fma(-a.y, t.x, sti));
        }
    }
    block_sum4x3(ss, str, sti, red);
    const double alpha = Sl[j].x;
    const double gamma = brk ? 0.0 : sqrt(fmax(alpha - ss, 0.0));
    int still = 1;
    if (j >= 1) {
        // complete column j - 1
        for (int i = tid; i < j; i += DC_STEP_BS) {
            double2 h = col[i];
            if (!brk) {
                const double2 a = Sl[i];
                h.x = fma(beta, a.x, h.x);
                h.y = fma(beta, a.y, h.y);
            }
            Hc[i] = h;
            col[i] = h;
        }
        if (tid == 0) {
            const double2 sub = make_double2(brk ? 0.0 : beta * gamma, 0.0);
            Hc[j] = sub;
            col[j] = sub;
        }
        __syncthreads();
        if (tid == 0) {
            const int c0 = j - 1;
            // the previous rotations in order; the running entry stays in
            // registers, so only the loads (independent of the chain) touch LDS
            double2 hi = col[0];
#pragma unroll 4
            for (int i = 0; i < c0; ++i) {
                const double2 hn = col[i + 1];
                const double2 ci = lc[i], si = ls[i];
                col[i] = make_double2(ci.x * hi.x - ci.y * hi.y + si.x * hn.x - si.y * hn.y,
                                      ci.x * hi.y + ci.y * hi.x + si.x * hn.y + si.y * hn.x);
                hi = make_double2(-(si.x * hi.x + si.y * hi.y) + (ci.x * hn.x + ci.y * hn.y),
                                  -(si.x * hi.y - si.y * hi.x) + (ci.x * hn.y - ci.y * hn.x));
            }
            col[c0] = hi;
            const double2 a = col[c0], b = col[c0 + 1];
            const double na = hypot(a.x, a.y), nb = hypot(b.x, b.y);
            const double rho = hypot(na, nb);
            double2 cj, sj;
            if (rho == 0.0) {
                cj = make_double2(1.0, 0.0);
                sj = make_double2(0.0, 0.0);
            } else if (na == 0.0) {
                cj = make_double2(0.0, 0.0);
                sj = make_double2(b.x / nb, -b.y / nb);
            } else {
                cj = make_double2(na / rho, 0.0);
                const double ux = a.x / na, uy = a.y / na;
                sj = make_double2((ux * b.x + uy * b.y) / rho, (uy * b.x - ux * b.y) / rho);
            }
            cs[(size_t)r * m + c0] = cj;
            sn[(size_t)r * m + c0] = sj;
            col[c0] = make_double2(cj.x * a.x + sj.x * b.x - sj.y * b.y, cj.x * a.y + sj.x * b.y + sj.y * b.x);
            col[c0 + 1] = make_double2(0.0, 0.0);
            double2* gv = gvec + (size_t)r * (m + 1);
            const double2 gj = gv[c0];
            const double2 gn = make_double2(-(sj.x * gj.x + sj.y * gj.y), -(sj.x * gj.y - sj.y * gj.x));
            gv[c0 + 1] = gn;
            gv[c0] = make_double2(cj.x * gj.x, cj.x * gj.y);
            const double res = hypot(gn.x, gn.y);
            const int it = iters[r] + 1;
            iters[r] = it;
            kdim[r] = j;
            // stop on convergence, a spent budget, the end of the Krylov space or a non-finite value
            still = (res > thr[r]) && it < maxit && (gamma > 0.0) && !brk;
            if (!still) active[r] = stop_mark;
            still_s = still;
        }
        __syncthreads();
        still = still_s;
        double2* Rc = H + (size_t)r * (m + 1) * m + (size_t)(j - 1) * (m + 1);
        for (int i = tid; i <= j; i += DC_STEP_BS) Rc[i] = col[i];
    } else if (!(gamma > 0.0)) {
        still = 0;
        if (tid == 0) active[r] = stop_mark;
    }
    if (j == m) still = 0;  // end of the cycle
    if (flags_out && tid == 0) flags_out[r] = still;
    if (!still) return;
    // column j and the update coefficients
    const double2 tau = Tl[j];
    const double ig = 1.0 / gamma;
    const double2 c = make_double2((tau.x - str) * ig, (tau.y - sti) * ig);
    const double2* Hr = Hraw + (size_t)r * (m + 1) * m;
    double2* Hj = Hraw + (size_t)r * (m + 1) * m + (size_t)j * (m + 1);
    // z_i = sum_l H[i, l] s_l over the Hessenberg band l >= i - 1, rows in
    // chunks of 64; wave w takes the columns l = w (mod 4), the four partial
    // sums are added in wave order
    for (int i0 = 0; i0 < jc; i0 += 64) {
        const int i = i0 + lane;
        double zr = 0.0, zi = 0.0;
        if (i < jc) {
            const int l0 = max(i - 1, 0);
            const int first = l0 + ((wv - l0) % 4 + 4) % 4;
#pragma unroll 8
            for (int l = first; l < j; l += 4) {
                const double2 h = Hr[(size_t)l * (m + 1) + i];
                const double2 a = Sl[l];
                zr += h.x * a.x - h.y * a.y;
                zi += h.x * a.y + h.y * a.x;
            }
        }
        zp[wv][lane] = make_double2(zr, zi);
        __syncthreads();
        if (wv == 0 && i < jc) {
            const double zx = ((zp[0][lane].x + zp[1][lane].x) + zp[2][lane].x) + zp[3][lane].x;
            const double zy = ((zp[0][lane].y + zp[1][lane].y) + zp[2][lane].y) + zp[3][lane].y;
            const double2 base = i < j ? Tl[i] : c;
            Hj[i] = make_double2((base.x - zx) * ig, (base.y - zy) * ig);
        }
        __syncthreads();
    }
}

// One pass over V_0..V_{j-1}: v_j = (vt - V s) / gamma (in place of the
// candidate) and w = (wt - V t - v_j c) / gamma; norm_out gets the partial of
// |w|^2 of each block.  Every block forms S, T, gamma and c itself from the
// projection partials, with the step block's sums in the step block's order,
// so the step's Hessenberg work runs beside the update instead of before it.
template <class TV>
__device__ __forceinline__ void dc_update(int r, int bx, int nu, TV* __restrict__ V, size_t ldv, int nr, int j, int m,
                                          int ns, const double2* __restrict__ partP,
                                          const double2* __restrict__ partQ, const double* __restrict__ hnorm,
                                          double2* __restrict__ W, size_t ldw, int n, double* __restrict__ norm_out,
                                          const int* __restrict__ active, TV* __restrict__ xt, int xw,
                                          double2* __restrict__ lds)
{
    if (!active[r]) return;
    const size_t L = (size_t)m + 1;
    double2* sl = lds;
    double2* tl = lds + L;
    double* red = reinterpret_cast<double*>(lds + 2 * L);
    const int jc = j + 1, tid = threadIdx.x;
    for (int i = tid; i < jc; i += BS) {
        double pr = 0.0, pi = 0.0, qr = 0.0, qi = 0.0;
#pragma unroll 8
        for (int b = 0; b < ns; ++b) {
            const size_t o = ((size_t)r * ns + b) * jc + i;
            const double2 p = partP[o];
            pr += p.x;
            pi += p.y;
            const double2 t = partQ[o];
            qr += t.x;
            qi += t.y;
        }
        sl[i] = make_double2(pr, pi);
        tl[i] = make_double2(qr, qi);
    }
    const double beta = j >= 1 ? hnorm[r] : 1.0;
    // this thread's candidate rows, loaded while the coefficients are formed
    const int q = bx * BS + threadIdx.x;
    TV* vj = V + ((size_t)j * nr + r) * ldv;
    double2 v = make_double2(0.0, 0.0), w = make_double2(0.0, 0.0);
    if (q < n) {
        v = ld2(vj + q);
        w = W[(size_t)r * ldw + q];
    }
    __syncthreads();
    if (!(beta > 0.0)) return;  // the previous step ended the Krylov space
    double ss = 0.0, str = 0.0, sti = 0.0;
    for (int i = tid; i < j; i += BS) {
        const double2 a = sl[i], t = tl[i];
        ss = fma(a.x, a.x, fma(a.y, a.y, ss));
        str = fma(a.x, t.x, fma(a.y, t.y, str));
        sti = fma(a.x, t.y, fma(-a.y, t.x, sti));
    }
    block_sum4x3(ss, str, sti, red);
    const double gamma = sqrt(fmax(sl[j].x - ss, 0.0));
    if (!(gamma > 0.0)) return;
    const double ig = 1.0 / gamma;
    const double2 tau = tl[j];
    const double2 c = make_double2((tau.x - str) * ig, (tau.y - sti) * ig);
    double nn[1] = {0.0};
    if (q < n) {
        for (int i = 0; i < j; ++i) {
            const double2 b = ld2(V + ((size_t)i * nr + r) * ldv + q);
            const double2 a = sl[i], t = tl[i];
            v.x -= a.x * b.x - a.y * b.y;
            v.y -= a.x * b.y + a.y * b.x;
            w.x -= t.x * b.x - t.y * b.y;
            w.y -= t.x * b.y + t.y * b.x;
        }
        v = make_double2(v.x * ig, v.y * ig);
        const double2 vc = cmul2(v, c);
        w = make_double2((w.x - vc.x) * ig, (w.y - vc.y) * ig);
        st2(vj + q, v);
        W[(size_t)r * ldw + q] = w;
        if (xt) st2(xt + (size_t)q * xw + r, w);  // the next product's input (its reduction divides by |w|)
        nn[0] = fma(w.x, w.x, w.y * w.y);
    }
    block_sum<1>(nn, red + 12);
    if (threadIdx.x == 0) norm_out[r * nu + bx] = nn[0];
}

// beta = |w| from the update partials (every block sums them in the same
// order), V_{j+1} = w / beta (0 if beta = 0: the Krylov space ended); with xt,
// also the packed copy the next product reads (XT[q * xw + r], the stored
// value), and zeros in its padding columns nr <= r < xw (grid rows).
template <class TV>
__device__ __forceinline__ void dc_next(int r, int bx, const double2* __restrict__ W, size_t ldw, int n,
                                        const double* __restrict__ norm_part, int nu, TV* __restrict__ V, size_t ldv,
                                        double* __restrict__ hnorm, int* __restrict__ active, int nr,
                                        TV* __restrict__ xt, int xw)
{
    __shared__ double bsh;
    const int q = bx * BS + threadIdx.x;
    if (r >= nr) {
        if (q < n) st2(xt + (size_t)q * xw + r, make_double2(0.0, 0.0));
        return;
    }
    const int act = active[r];
    if (act != 1) {
        // a column marked stopping at this step: clear the mark (every block
        // of the column returns here, whether it reads the mark or the zero)
        if (act == STOPPING && bx == 0 && threadIdx.x == 0) active[r] = 0;
        return;
    }
    if (threadIdx.x < 64) {
        const double beta = dev::step_beta(norm_part + (size_t)r * nu, nu);
        if (threadIdx.x == 0) bsh = beta;
    }
    __syncthreads();
    const double beta = bsh;
    if (bx == 0 && threadIdx.x == 0) hnorm[r] = beta;
    if (q >= n) return;
    const double inv = dev::inv_beta(beta);
    const double2 w = W[(size_t)r * ldw + q];
    const double2 v = make_double2(w.x * inv, w.y * inv);
    st2(V + (size_t)r * ldv + q, v);
    if (xt) st2(xt + (size_t)q * xw + r, v);
}

// v_0 = r / |r| and g = |r| e_0 per active right-hand side; with xt, also the
// packed copy of v_0 for the first product (as k_dc_next).
template <class TV>
__global__ void k_start_cycle(const double2* __restrict__ R, size_t ldr, int n, int nr,
                              const double* __restrict__ rnorm, int m, TV* __restrict__ V, size_t ldv,
                              double2* __restrict__ gvec, const int* __restrict__ active, TV* __restrict__ xt, int xw)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (r >= nr) {
        if (q < n) st2(xt + (size_t)q * xw + r, make_double2(0.0, 0.0));
        return;
    }
    if (!active[r]) return;
    const double nv = rnorm[r];
    const double inv = nv > 0.0 ? 1.0 / nv : 0.0;
    if (q < n) {
        const double2 v = R[(size_t)r * ldr + q];
        const double2 u = make_double2(v.x * inv, v.y * inv);
        st2(V + (size_t)r * ldv + q, u);
        if (xt) st2(xt + (size_t)q * xw + r, u);
    }
    if (q <= m) gvec[(size_t)r * (m + 1) + q] = make_double2(q == 0 ? nv : 0.0, 0.0);
}


template <class TV>
__global__ void k_xupdate(const TV* __restrict__ V, size_t ldv, int nr, int n, int m, const double2* __restrict__ y,
                          const int* __restrict__ kdim, double2* __restrict__ X, size_t ldx)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (q >= n) return;
    const int k = kdim[r];
    if (k == 0) return;
    double2 x = X[(size_t)r * ldx + q];
    const double2* yr = y + (size_t)r * (m + 1);
    for (int i = 0; i < k; ++i) {
        const double2 c = yr[i];
        const double2 v = ld2(V + ((size_t)i * nr + r) * ldv + q);
        x.x += c.x * v.x - c.y * v.y;
        x.y += c.x * v.y + c.y * v.x;
    }
    X[(size_t)r * ldx + q] = x;
}

__global__ void k_axpby_res(const double2* __restrict__ B, size_t ldb, const double2* __restrict__ AX, size_t ldax,
                            int n, double2* __restrict__ R, size_t ldr)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (q >= n) return;
    const double2 b = B[(size_t)r * ldb + q], a = AX[(size_t)r * ldax + q];
    R[(size_t)r * ldr + q] = make_double2(b.x - a.x, b.y - a.y);
}

__global__ void k_add_64(const double2* __restrict__ D, size_t ldd, int n, double2* __restrict__ X, size_t ldx,
                         const int* __restrict__ active)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (q >= n || (active && !active[r])) return;
    const double2 d = D[(size_t)r * ldd + q];
    double2 x = X[(size_t)r * ldx + q];
    x.x += d.x;
    x.y += d.y;
    X[(size_t)r * ldx + q] = x;
}

// ---------------------------------------------------------------------------
// Far field in the host medium: F(th) = e^{i pi/4}/sqrt(8 pi k0)
//   sum_j sigma_j [w_j + i k0 (xh.n_j) u_j] h_j e^{-i k0 xh.c_j} sinc(k0 h_j xh.t_j/2)
// (large-|x| form of G, element integral exact).  One block per direction.
// ---------------------------------------------------------------------------
constexpr int FF_NR = 8;

__global__ __launch_bounds__(BS) void k_farfield(const char* __restrict__ g, GeomLayout L, int N, int n_if,
                                                 const double2* __restrict__ X, size_t ldx, int nrhs,
                                                 AngleChunk dirs, double2* __restrict__ F, size_t ldf)
{
    __shared__ double lds[4 * 2 * FF_NR];
    const int d = blockIdx.x;
    const int r0 = blockIdx.y * FF_NR;
    const ElemRec* el = tab<ElemRec>(g, L.elem);
    const int* elif = tab<int>(g, L.elif);
    const int* sigma = tab<int>(g, L.sigma);
    const double k0 = tab<DomConst>(g, L.dom)[0].k[0];
    double sx, cx;
    sincos(dirs.v[d], &sx, &cx);
    double acc[2 * FF_NR];
#pragma unroll
    for (int k = 0; k < 2 * FF_NR; ++k) acc[k] = 0.0;
    for (int e = threadIdx.x; e < N; e += BS) {
        const int sg = sigma[elif[e]];  // domain 0 row of the sigma table
        if (sg == 0) continue;
        const ElemRec E = el[e];
        const double a = 0.5 * k0 * E.h * (cx * E.tx + sx * E.ty);
        const double sinc = (a == 0.0) ? 1.0 : sin(a) / a;
        double sp, cp;
        sincos(-k0 * (cx * E.cx + sx * E.cy), &sp, &cp);
        const double f = sg * E.h * sinc;
        const double fr = f * cp, fi = f * sp;           // sigma h sinc e^{-i k0 xh.c}
        const double gk = k0 * (cx * E.nx + sx * E.ny);  // i gk u
#pragma unroll
        for (int k = 0; k < FF_NR; ++k) {
            const int r = r0 + k;
            if (r < nrhs) {
                const double2 u = X[(size_t)r * ldx + e], w = X[(size_t)r * ldx + N + e];
                const double tr = w.x - gk * u.y, ti = w.y + gk * u.x;
                acc[2 * k] += fr * tr - fi * ti;
                acc[2 * k + 1] += fr * ti + fi * tr;
            }
        }
    }
    block_sum<2 * FF_NR>(acc, lds);
    if (threadIdx.x == 0) {
        const double pre = 1.0 / sqrt(8.0 * 3.14159265358979323846 * k0);
        const double c4 = 0.70710678118654752440;  // e^{i pi/4} = (1 + i)/sqrt2
        for (int k = 0; k < FF_NR; ++k) {
            const int r = r0 + k;
            if (r < nrhs) {
                const double xr = acc[2 * k] * pre, xi = acc[2 * k + 1] * pre;
                F[(size_t)r * ldf + d] = make_double2(c4 * (xr - xi), c4 * (xr + xi));
            }
        }
    }
}

// ---------------------------------------------------------------------------
// One Arnoldi step of up to MAX_FUSED problems in each launch (fused
// multi-instance steps): the problems' block ranges follow each other in a
// one-dimensional grid, and every block runs the single-problem body above
// with its problem's buffers, so each problem's arithmetic and reduction order
// are the same alone or fused.  All problems share the step index j and the
// restart length m (they run their cycles in step); a problem absent from a
// launch is simply not in the set.
// ---------------------------------------------------------------------------
struct ArnProb {
    void* V;
    double2* W;
    size_t ldv, ldw;
    double2 *partP, *partQ, *Hraw, *H, *cs, *sn, *gvec;
    double *hnorm, *norm_part;
    const double* thr;
    int *iters, *kdim, *active, *flags_out;
    void* xt;
    int nr, n, maxit, xw;
    int ns, rcp, nu;  // projection row chunks, padded (right-hand side, chunk) pairs, update blocks
    int b0[4];        // first block of this problem in the projection, step, update and next launches
};
// NP: capacity of the set.  A lone problem launches with NP = 1, whose
// descriptor (about 220 bytes of kernel arguments) is an eighth of the fused
// one's, and whose blocks need no search for their problem.
template <int NP>
struct ArnSet {
    int np;
    ArnProb p[NP];
};

// the problem whose block range of launch k holds block b
template <int NP>
__device__ __forceinline__ int set_problem(const ArnSet<NP>& S, int k, int b)
{
    if constexpr (NP == 1) {
        return 0;
    } else {
        int i = 0;
        while (i + 1 < S.np && b >= S.p[i + 1].b0[k]) ++i;
        return i;
    }
}

template <int BATCH, bool HASW, class TV, int NP>
__global__ __launch_bounds__(BS) void k_dc_dots(const ArnSet<NP> S, int jc, int rpt)
{
    const ArnProb& P = S.p[set_problem(S, 0, blockIdx.x)];
    dc_dots<BATCH, HASW, TV>((int)blockIdx.x - P.b0[0], static_cast<const TV*>(P.V), P.ldv, P.nr, jc, P.W, P.ldw, P.n,
                             rpt, P.ns, P.rcp, P.partP, HASW ? P.partQ : nullptr, P.active);
}

// Step blocks first (one per right-hand side: the Hessenberg column, the
// rotations, the stopping decision), then the update blocks (nu per
// right-hand side); at the last step of a cycle only the step blocks.
static_assert(DC_STEP_BS == BS, "step and update blocks share one launch");
template <class TV, int NP>
__global__ __launch_bounds__(BS) void k_dc_update(const ArnSet<NP> S, int j, int m, bool last)
{
    extern __shared__ double2 arn_lds[];
    const ArnProb& P = S.p[set_problem(S, 2, blockIdx.x)];
    const int b = (int)blockIdx.x - P.b0[2];
    if (b < P.nr) {
        dc_step(b, P.nr, j, m, P.ns, P.partP, last ? nullptr : P.partQ, P.Hraw, P.H, P.cs, P.sn, P.gvec, P.hnorm,
                P.thr, P.maxit, P.iters, P.kdim, P.active, P.flags_out, arn_lds);
        return;
    }
    const int u = b - P.nr;
    dc_update<TV>(u / P.nu, u % P.nu, P.nu, static_cast<TV*>(P.V), P.ldv, P.nr, j, m, P.ns, P.partP, P.partQ,
                  P.hnorm, P.W, P.ldw, P.n, P.norm_part, P.active, static_cast<TV*>(P.xt), P.xw, arn_lds);
}

template <class TV, int NP>
__global__ __launch_bounds__(BS) void k_dc_next(const ArnSet<NP> S, int jc)
{
    const ArnProb& P = S.p[set_problem(S, 3, blockIdx.x)];
    const int b = (int)blockIdx.x - P.b0[3];
    dc_next<TV>(b / P.nu, b % P.nu, P.W, P.ldw, P.n, P.norm_part, P.nu,
                static_cast<TV*>(P.V) + (size_t)jc * P.nr * P.ldv, P.ldv, P.hnorm, P.active, P.nr,
                static_cast<TV*>(P.xt), P.xw);
}

}  // namespace

hipError_t launch_rhs(const char* g, const GeomLayout& L, int N, const double* angles, int nang, double2* B,
                      size_t ldb, hipStream_t s)
{
    for (int a0 = 0; a0 < nang; a0 += ANGLE_CHUNK) {
        const int na = std::min(ANGLE_CHUNK, nang - a0);
        AngleChunk c{};
        for (int k = 0; k < na; ++k) c.v[k] = angles[a0 + k];
        hipLaunchKernelGGL(k_rhs, dim3((N + 127) / 128, na), dim3(128), 0, s, g, L, N, c, na, B + (size_t)a0 * ldb,
                           ldb);
    }
    return hipGetLastError();
}

hipError_t launch_col_norms(const double2* X, size_t ldx, int n, int nr, double* partial, double* out,
                            hipStream_t s)
{
    const int nblk = std::min(64, (n + BS - 1) / BS);
    hipLaunchKernelGGL(k_col_norm_partial, dim3(nblk, nr), dim3(BS), 0, s, X, ldx, n, partial);
    hipLaunchKernelGGL(k_col_norm_finish, dim3((nr + 63) / 64), dim3(64), 0, s, partial, nblk, nr, out);
    return hipGetLastError();
}

// Shape of the projection kernel: rows per block (a multiple of BS) and basis
// vectors per block (4, 8 or 16); BEM_DOT_CFG="rows,batch" overrides it
// (tuning).  Measured on gfx950: 2048 rows of 4 vectors against 512 rows
// gives kite4096 (16 right-hand sides) 531 against 522 solves/s, kite16384
// (64, FP32 products) 94.4 against 93.1, the served stream 473 against 458
// mixed solves/s; 4096 rows 529, 8 vectors per block 496.
struct DotCfg {
    int rows, batch;
};

DotCfg dot_cfg()
{
    DotCfg c{2048, 4};
    if (const char* e = getenv("BEM_DOT_CFG")) {
        int a = 0, b = 0;
        if (sscanf(e, "%d,%d", &a, &b) == 2 && a >= BS && a <= 16384 && a % BS == 0 && (b == 4 || b == 8 || b == 16))
            c = {a, b};
    }
    return c;
}

int update_blocks(int n) { return (n + BS - 1) / BS; }

int arnoldi_blocks(int n) { return std::max((n + BS - 1) / BS, (n + dot_cfg().rows - 1) / dot_cfg().rows); }

namespace {

template <bool HASW, class TV, int NP>
void launch_dc_dots(const DotCfg& c, const ArnSet<NP>& S, int nblocks, int jc, hipStream_t s)
{
    const int rpt = c.rows / BS;
    if (c.batch == 4)
        hipLaunchKernelGGL((k_dc_dots<4, HASW, TV, NP>), dim3(nblocks), dim3(BS), 0, s, S, jc, rpt);
    else if (c.batch == 16)
        hipLaunchKernelGGL((k_dc_dots<16, HASW, TV, NP>), dim3(nblocks), dim3(BS), 0, s, S, jc, rpt);
    else
        hipLaunchKernelGGL((k_dc_dots<8, HASW, TV, NP>), dim3(nblocks), dim3(BS), 0, s, S, jc, rpt);
}

template <class TV, int NP>
hipError_t launch_arnoldi_kernels(const DotCfg& dc, const ArnSet<NP>& S, const int nb[4], int j, int m,
                                  hipStream_t s)
{
    const int jc = j + 1;
    const bool last = j == m;
    // problems whose products read packed right-hand sides normalise v_j in
    // the product of step j; at the last step, which has no product, here
    if (last && nb[3] > 0) hipLaunchKernelGGL((k_dc_next<TV, NP>), dim3(nb[3]), dim3(BS), 0, s, S, j);
    if (last)
        launch_dc_dots<false, TV>(dc, S, nb[0], jc, s);
    else
        launch_dc_dots<true, TV>(dc, S, nb[0], jc, s);
    hipLaunchKernelGGL((k_dc_update<TV, NP>), dim3(nb[2]), dim3(BS), arn_lds_elems(m) * sizeof(double2), s, S, j, m,
                       last);
    if (!last && nb[3] > 0) hipLaunchKernelGGL((k_dc_next<TV, NP>), dim3(nb[3]), dim3(BS), 0, s, S, jc);
    return hipGetLastError();
}

template <class TV>
hipError_t launch_arnoldi_t(const ArnoldiArgs* a, int np, int j, hipStream_t s)
{
    const DotCfg dc = dot_cfg();
    const int m = a[0].m;
    const int jc = j + 1;
    ArnSet<MAX_FUSED> S{};
    S.np = np;
    int nb[4] = {0, 0, 0, 0};
    for (int k = 0; k < np; ++k) {
        const ArnoldiArgs& A = a[k];
        ArnProb& P = S.p[k];
        P.V = A.V;
        P.W = A.W;
        P.ldv = A.ldv;
        P.ldw = A.ldw;
        P.partP = A.partP;
        P.partQ = A.partQ;
        P.Hraw = A.Hraw;
        P.H = A.H;
        P.cs = A.cs;
        P.sn = A.sn;
        P.gvec = A.gvec;
        P.hnorm = A.hnorm;
        P.norm_part = A.norm_part;
        P.thr = A.thr;
        P.iters = A.iters;
        P.kdim = A.kdim;
        P.active = A.active;
        P.flags_out = A.flags_out;
        P.xt = A.xt;
        P.nr = A.nr;
        P.n = A.n;
        P.maxit = A.maxit;
        P.xw = A.xw;
        P.ns = (A.n + dc.rows - 1) / dc.rows;  // row chunks of the projection kernel
        P.rcp = (A.nr * P.ns + 7) / 8 * 8;
        P.nu = update_blocks(A.n);              // blocks of the update kernel
        // projection, (unused), step + update, normalisation blocks; the
        // normalisation of a problem with packed product inputs runs only at
        // the last step (before the projection)
        const bool packed = A.xt != nullptr;
        const int counts[4] = {P.rcp * ((jc + dc.batch - 1) / dc.batch), 0, A.nr + (j == m ? 0 : P.nu * A.nr),
                               (j == m) == packed ? P.nu * A.nr : 0};
        for (int q = 0; q < 4; ++q) {
            P.b0[q] = nb[q];
            nb[q] += counts[q];
        }
    }
    if (np == 1) {
        ArnSet<1> S1{};
        S1.np = 1;
        S1.p[0] = S.p[0];
        return launch_arnoldi_kernels<TV>(dc, S1, nb, j, m, s);
    }
    return launch_arnoldi_kernels<TV>(dc, S, nb, j, m, s);
}

}  // namespace

hipError_t launch_arnoldi(const ArnoldiArgs& a, int j, hipStream_t s) { return launch_arnoldi_set(&a, 1, j, s); }

hipError_t launch_arnoldi_set(const ArnoldiArgs* a, int np, int j, hipStream_t s)
{
    if (np < 1 || np > MAX_FUSED) return hipErrorInvalidValue;
    for (int k = 1; k < np; ++k)
        if (a[k].v32 != a[0].v32 || a[k].m != a[0].m) return hipErrorInvalidValue;
    if (a[0].v32) return launch_arnoldi_t<float2>(a, np, j, s);
    return launch_arnoldi_t<double2>(a, np, j, s);
}

namespace {

template <class TV>
hipError_t start_cycle_t(const double2* R, size_t ldr, int n, int nr, const double* rnorm, int m, TV* V, size_t ldv,
                         double2* gvec, const int* active, TV* xt, int xw, hipStream_t s)
{
    const int len = std::max(n, m + 1);
    hipLaunchKernelGGL((k_start_cycle<TV>), dim3((len + BS - 1) / BS, xt ? xw : nr), dim3(BS), 0, s, R, ldr, n, nr,
                       rnorm, m, V, ldv, gvec, active, xt, xw);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_start_cycle(const double2* R, size_t ldr, int n, int nr, const double* rnorm, int m,
                              double2* V, size_t ldv, double2* gvec, const int* active, double2* xt, int xw,
                              hipStream_t s)
{
    return start_cycle_t(R, ldr, n, nr, rnorm, m, V, ldv, gvec, active, xt, xw, s);
}

hipError_t launch_start_cycle(const double2* R, size_t ldr, int n, int nr, const double* rnorm, int m,
                              float2* V, size_t ldv, double2* gvec, const int* active, float2* xt, int xw,
                              hipStream_t s)
{
    return start_cycle_t(R, ldr, n, nr, rnorm, m, V, ldv, gvec, active, xt, xw, s);
}

hipError_t launch_backsolve(int nr, int m, const double2* H, const double2* gvec, const int* kdim, double2* y,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_backsolve_wave, dim3(nr), dim3(64), (size_t)m * sizeof(double2), s, nr, m, H, gvec, kdim,
                       y);
    return hipGetLastError();
}

hipError_t launch_xupdate(const double2* V, size_t ldv, int nr, int n, int m, const double2* y, const int* kdim,
                          double2* X, size_t ldx, hipStream_t s)
{
    hipLaunchKernelGGL((k_xupdate<double2>), dim3((n + BS - 1) / BS, nr), dim3(BS), 0, s, V, ldv, nr, n, m, y, kdim, X,
                       ldx);
    return hipGetLastError();
}

hipError_t launch_xupdate(const float2* V, size_t ldv, int nr, int n, int m, const double2* y, const int* kdim,
                          double2* X, size_t ldx, hipStream_t s)
{
    hipLaunchKernelGGL((k_xupdate<float2>), dim3((n + BS - 1) / BS, nr), dim3(BS), 0, s, V, ldv, nr, n, m, y, kdim, X,
                       ldx);
    return hipGetLastError();
}

hipError_t launch_axpby_res(const double2* B, size_t ldb, const double2* AX, size_t ldax, int n, int nr,
                            double2* R, size_t ldr, hipStream_t s)
{
    hipLaunchKernelGGL(k_axpby_res, dim3((n + BS - 1) / BS, nr), dim3(BS), 0, s, B, ldb, AX, ldax, n, R, ldr);
    return hipGetLastError();
}

hipError_t launch_add_f64(const double2* D, size_t ldd, int n, int nr, double2* X, size_t ldx, const int* active,
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_add_64, dim3((n + BS - 1) / BS, nr), dim3(BS), 0, s, D, ldd, n, X, ldx, active);
    return hipGetLastError();
}

hipError_t launch_farfield(const char* g, const GeomLayout& L, int N, int n_if, int n_dom, const double2* X,
                           size_t ldx, int nrhs, const double* dirs, int ndir, double2* F, size_t ldf, hipStream_t s)
{
    (void)n_dom;
    for (int d0 = 0; d0 < ndir; d0 += ANGLE_CHUNK) {
        const int nd = std::min(ANGLE_CHUNK, ndir - d0);
        AngleChunk c{};
        for (int k = 0; k < nd; ++k) c.v[k] = dirs[d0 + k];
        hipLaunchKernelGGL(k_farfield, dim3(nd, (nrhs + FF_NR - 1) / FF_NR), dim3(BS), 0, s, g, L, N, n_if, X, ldx,
                           nrhs, c, F + d0, ldf);
    }
    return hipGetLastError();
}

}  // namespace bemk
