// linalg.hip -- right-hand sides and the batched GMRES(m) building blocks (Sec. 3.2: GMRES on A itself, x0 = 0),
// plus the far-field output step.
//
// Layouts: matrices column-major; a block of vectors is column-major with one
// column per right-hand side.  The Krylov basis of all right-hand sides is
// V[(i * nr + r) * ldv + q] (basis vector i of right-hand side r, row q).
// All reductions run in a fixed order, so repeated runs are bitwise equal.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "launch.h"

namespace bemk {

namespace {

constexpr int BS = 256;        // threads per block
constexpr int DOT_BATCH = 8;   // basis vectors reduced together

template <class T>
__device__ __forceinline__ const T* tab(const char* g, size_t off) { return reinterpret_cast<const T*>(g + off); }

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

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

// partial[(r * nblk + blk) * jcount + i] = sum over the block's rows of conj(V_i) W
__global__ __launch_bounds__(BS) void k_dots(const double2* __restrict__ V, size_t ldv, int nr, int jcount,
                                             const double2* __restrict__ W, size_t ldw, int n,
                                             double2* __restrict__ part, const int* __restrict__ active)
{
    __shared__ double lds[4 * 2 * DOT_BATCH];
    const int r = blockIdx.y;
    if (!active[r]) return;
    const int q = blockIdx.x * BS + threadIdx.x;
    double2 w = make_double2(0.0, 0.0);
    if (q < n) w = W[(size_t)r * ldw + q];
    for (int i0 = 0; i0 < jcount; i0 += DOT_BATCH) {
        double acc[2 * DOT_BATCH];
#pragma unroll
        for (int b = 0; b < DOT_BATCH; ++b) {
            const int i = i0 + b;
            double2 v = make_double2(0.0, 0.0);
            if (i < jcount && q < n) v = V[((size_t)i * nr + r) * ldv + q];
            acc[2 * b] = fma(v.x, w.x, v.y * w.y);      // Re conj(v) w
            acc[2 * b + 1] = fma(v.x, w.y, -v.y * w.x); // Im conj(v) w
        }
        block_sum<2 * DOT_BATCH>(acc, lds);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int b = 0; b < DOT_BATCH; ++b)
                if (i0 + b < jcount)
                    part[((size_t)r * gridDim.x + blockIdx.x) * jcount + i0 + b] =
                        make_double2(acc[2 * b], acc[2 * b + 1]);
        }
    }
}

__global__ void k_dots_reduce(const double2* __restrict__ part, int nblk, int nr, int jcount,
                              double2* __restrict__ h, const int* __restrict__ active)
{
    const int r = blockIdx.x;
    if (!active[r]) return;
    for (int i = threadIdx.x; i < jcount; i += blockDim.x) {
        double sr = 0.0, si = 0.0;
        for (int b = 0; b < nblk; ++b) {
            const double2 v = part[((size_t)r * nblk + b) * jcount + i];
            sr += v.x;
            si += v.y;
        }
        h[(size_t)r * 1024 + i] = make_double2(sr, si);
    }
}

// W -= sum_i h_i V_i ; optional per-block partial sums of |W|^2
__global__ __launch_bounds__(BS) void k_update(const double2* __restrict__ V, size_t ldv, int nr, int jcount,
                                               const double2* __restrict__ h, double2* __restrict__ W, size_t ldw,
                                               int n, const int* __restrict__ active,
                                               double* __restrict__ norm_part)
{
    __shared__ double lds[4];
    const int r = blockIdx.y;
    if (!active[r]) return;
    const int q = blockIdx.x * BS + threadIdx.x;
    double acc[1] = {0.0};
    if (q < n) {
        double2 w = W[(size_t)r * ldw + q];
        const double2* hr = h + (size_t)r * 1024;
        for (int i = 0; i < jcount; ++i) {
            const double2 c = hr[i];
            const double2 v = V[((size_t)i * nr + r) * ldv + q];
            w.x -= c.x * v.x - c.y * v.y;
            w.y -= c.x * v.y + c.y * v.x;
        }
        W[(size_t)r * ldw + q] = w;
        acc[0] = fma(w.x, w.x, w.y * w.y);
    }
    if (norm_part) {
        block_sum<1>(acc, lds);
        if (threadIdx.x == 0) norm_part[r * gridDim.x + blockIdx.x] = acc[0];
    }
}

// H[:, j] = h1 + h2 (two Gram-Schmidt passes), H[j+1, j] = ||w||
__global__ void k_arnoldi_finish(int nr, int j, int m, const double2* __restrict__ h1,
                                 const double2* __restrict__ h2, const double* __restrict__ norm_part, int nblk,
                                 double2* __restrict__ H, double* __restrict__ hnorm, const int* __restrict__ active)
{
    const int r = blockIdx.x;
    if (!active[r]) return;
    double2* Hr = H + (size_t)r * (m + 1) * m;
    for (int i = threadIdx.x; i <= j; i += blockDim.x) {
        const double2 a = h1[(size_t)r * 1024 + i], b = h2[(size_t)r * 1024 + i];
        Hr[i + (size_t)j * (m + 1)] = make_double2(a.x + b.x, a.y + b.y);
    }
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int b = 0; b < nblk; ++b) s += norm_part[r * nblk + b];
        const double nv = sqrt(s);
        Hr[j + 1 + (size_t)j * (m + 1)] = make_double2(nv, 0.0);
        hnorm[r] = nv;
    }
}

__global__ void k_scale_into(const double2* __restrict__ W, size_t ldw, int n, const double* __restrict__ hnorm,
                             double2* __restrict__ V, size_t ldv, int nr, const int* __restrict__ active)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (q >= n || !active[r]) return;
    const double nv = hnorm[r];
    const double inv = nv > 0.0 ? 1.0 / nv : 0.0;
    const double2 w = W[(size_t)r * ldw + q];
    V[(size_t)r * ldv + q] = make_double2(w.x * inv, w.y * inv);
}

// Apply the earlier rotations to column j of H, make the rotation that zeroes
// H[j+1, j], update g and the residual estimate |g[j+1]|.
__global__ void k_givens(int nr, int j, int m, double2* __restrict__ H, double2* __restrict__ cs,
                         double2* __restrict__ sn, double2* __restrict__ gvec, double* __restrict__ resid,
                         const int* __restrict__ active)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr || !active[r]) return;
    double2* Hc = H + (size_t)r * (m + 1) * m + (size_t)j * (m + 1);
    double2* c = cs + (size_t)r * m;
    double2* s = sn + (size_t)r * m;
    double2* gv = gvec + (size_t)r * (m + 1);
    for (int i = 0; i < j; ++i) {
        const double2 hi = Hc[i], hn = Hc[i + 1];
        const double2 ci = c[i], si = s[i];
        // [hi; hn] <- [c s; -conj(s) conj(c)] [hi; hn]
        const double2 t = make_double2(ci.x * hi.x - ci.y * hi.y + si.x * hn.x - si.y * hn.y,
                                       ci.x * hi.y + ci.y * hi.x + si.x * hn.y + si.y * hn.x);
        const double2 u = make_double2(-(si.x * hi.x + si.y * hi.y) + (ci.x * hn.x + ci.y * hn.y),
                                       -(si.x * hi.y - si.y * hi.x) + (ci.x * hn.y - ci.y * hn.x));
        Hc[i] = t;
        Hc[i + 1] = u;
    }
    const double2 a = Hc[j], b = Hc[j + 1];
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
        // c = |a|/rho, s = (a/|a|) conj(b) / rho
        cj = make_double2(na / rho, 0.0);
        const double ux = a.x / na, uy = a.y / na;
        sj = make_double2((ux * b.x + uy * b.y) / rho, (uy * b.x - ux * b.y) / rho);
    }
    c[j] = cj;
    s[j] = sj;
    Hc[j] = make_double2(cj.x * a.x + sj.x * b.x - sj.y * b.y, cj.x * a.y + sj.x * b.y + sj.y * b.x);
    Hc[j + 1] = make_double2(0.0, 0.0);
    const double2 gj = gv[j];
    // g[j+1] = -conj(s) g[j]; g[j] = c g[j]
    gv[j + 1] = make_double2(-(sj.x * gj.x + sj.y * gj.y), -(sj.x * gj.y - sj.y * gj.x));
    gv[j] = make_double2(cj.x * gj.x, cj.x * gj.y);
    resid[r] = hypot(gv[j + 1].x, gv[j + 1].y);
}


// Column j of the Hessenberg matrix (h1 + h2 from the two Gram-Schmidt passes,
// ||w|| below the diagonal), then the Givens update of that column and of g:
// one wave per right-hand side; the column and the rotations sit in LDS and
// lane 0 applies the rotations in order.
__global__ __launch_bounds__(64) void k_arnoldi_givens(int nr, int j, int m, const double2* __restrict__ h1,
                                                       const double2* __restrict__ h2,
                                                       const double* __restrict__ norm_part, int nblk,
                                                       double2* __restrict__ H, double2* __restrict__ cs,
                                                       double2* __restrict__ sn, double2* __restrict__ gvec,
                                                       double* __restrict__ hnorm, double* __restrict__ resid,
                                                       const int* __restrict__ active)
{
    __shared__ double2 col[1024 + 1];
    __shared__ double2 lc[1024], ls[1024];
    const int r = blockIdx.x;
    if (!active[r]) return;
    const int lane = threadIdx.x;
    double2* Hc = H + (size_t)r * (m + 1) * m + (size_t)j * (m + 1);
    for (int i = lane; i <= j; i += 64) {
        const double2 a = h1[(size_t)r * 1024 + i], b = h2[(size_t)r * 1024 + i];
        col[i] = make_double2(a.x + b.x, a.y + b.y);
    }
    for (int i = lane; i < j; i += 64) {
        lc[i] = cs[(size_t)r * m + i];
        ls[i] = sn[(size_t)r * m + i];
    }
    double part = 0.0;
    for (int b = lane; b < nblk; b += 64) part += norm_part[r * nblk + b];
    // fixed-order sum over the wave
    __shared__ double red[64];
    red[lane] = part;
    __syncthreads();
    if (lane == 0) {
        double sum = 0.0;
        for (int k = 0; k < 64; ++k) sum += red[k];
        const double nv = sqrt(sum);
        hnorm[r] = nv;
        col[j + 1] = make_double2(nv, 0.0);
        for (int i = 0; i < j; ++i) {
            const double2 hi = col[i], hn = col[i + 1];
            const double2 ci = lc[i], si = ls[i];
            col[i] = make_double2(ci.x * hi.x - ci.y * hi.y + si.x * hn.x - si.y * hn.y,
                                  ci.x * hi.y + ci.y * hi.x + si.x * hn.y + si.y * hn.x);
            col[i + 1] = make_double2(-(si.x * hi.x + si.y * hi.y) + (ci.x * hn.x + ci.y * hn.y),
                                      -(si.x * hi.y - si.y * hi.x) + (ci.x * hn.y - ci.y * hn.x));
        }
        const double2 a = col[j], b = col[j + 1];
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
        cs[(size_t)r * m + j] = cj;
        sn[(size_t)r * m + j] = sj;
        col[j] = make_double2(cj.x * a.x + sj.x * b.x - sj.y * b.y, cj.x * a.y + sj.x * b.y + sj.y * b.x);
        col[j + 1] = make_double2(0.0, 0.0);
        double2* gv = gvec + (size_t)r * (m + 1);
        const double2 gj = gv[j];
        const double2 gn = make_double2(-(sj.x * gj.x + sj.y * gj.y), -(sj.x * gj.y - sj.y * gj.x));
        gv[j + 1] = gn;
        gv[j] = make_double2(cj.x * gj.x, cj.x * gj.y);
        resid[r] = hypot(gn.x, gn.y);
    }
    __syncthreads();
    for (int i = lane; i <= j + 1; i += 64) Hc[i] = col[i];
}

// y = H(0:k, 0:k)^{-1} g(0:k), column-oriented back substitution: one wave per
// right-hand side, g in LDS; step i divides by H(i, i) and removes column i
// from the rows above it (lanes over rows).
__global__ __launch_bounds__(64) void k_backsolve_wave(int nr, int m, const double2* __restrict__ H,
                                                       const double2* __restrict__ gvec,
                                                       const int* __restrict__ kdim, double2* __restrict__ y)
{
    __shared__ double2 g[1024];
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
            y[(size_t)r * 1024 + i] = yi;
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

__global__ void k_start_cycle(const double2* __restrict__ R, size_t ldr, int n, int nr,
                              const double* __restrict__ rnorm, int m, double2* __restrict__ V, size_t ldv,
                              double2* __restrict__ gvec, const int* __restrict__ active)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (!active[r]) return;
    const double nv = rnorm[r];
    const double inv = nv > 0.0 ? 1.0 / nv : 0.0;
    if (q < n) {
        const double2 v = R[(size_t)r * ldr + q];
        V[(size_t)r * ldv + q] = make_double2(v.x * inv, v.y * inv);
    }
    if (q <= m) gvec[(size_t)r * (m + 1) + q] = make_double2(q == 0 ? nv : 0.0, 0.0);
}

__global__ void k_backsolve(int nr, int m, const double2* __restrict__ H, const double2* __restrict__ gvec,
                            const int* __restrict__ kdim, double2* __restrict__ y)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    const int k = kdim[r];
    const double2* Hr = H + (size_t)r * (m + 1) * m;
    double2* yr = y + (size_t)r * 1024;
    for (int i = k - 1; i >= 0; --i) {
        double sr = gvec[(size_t)r * (m + 1) + i].x, si = gvec[(size_t)r * (m + 1) + i].y;
        for (int p = i + 1; p < k; ++p) {
            const double2 h = Hr[i + (size_t)p * (m + 1)], v = yr[p];
            sr -= h.x * v.x - h.y * v.y;
            si -= h.x * v.y + h.y * v.x;
        }
        const double2 d = Hr[i + (size_t)i * (m + 1)];
        const double den = d.x * d.x + d.y * d.y;
        yr[i] = den > 0.0 ? make_double2((sr * d.x + si * d.y) / den, (si * d.x - sr * d.y) / den)
                          : make_double2(0.0, 0.0);
    }
}

__global__ void k_xupdate(const double2* __restrict__ V, size_t ldv, int nr, int n, const double2* __restrict__ y,
                          const int* __restrict__ kdim, double2* __restrict__ X, size_t ldx)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (q >= n) return;
    const int k = kdim[r];
    if (k == 0) return;
    double2 x = X[(size_t)r * ldx + q];
    const double2* yr = y + (size_t)r * 1024;
    for (int i = 0; i < k; ++i) {
        const double2 c = yr[i];
        const double2 v = V[((size_t)i * nr + r) * ldv + q];
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

__global__ void k_cast_64_32(const double2* __restrict__ X, size_t ldx, int n, float2* __restrict__ Y, size_t ldy)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (q >= n) return;
    const double2 v = X[(size_t)r * ldx + q];
    Y[(size_t)r * ldy + q] = make_float2((float)v.x, (float)v.y);
}

__global__ void k_cast_32_64(const float2* __restrict__ X, size_t ldx, int n, double2* __restrict__ Y, size_t ldy)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (q >= n) return;
    const float2 v = X[(size_t)r * ldx + q];
    Y[(size_t)r * ldy + q] = make_double2((double)v.x, (double)v.y);
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

hipError_t launch_dots(const double2* V, size_t ldv, int nr, int jcount, const double2* W, size_t ldw, int n,
                       double2* partial, double2* h, const int* active, hipStream_t s)
{
    const int nblk = (n + BS - 1) / BS;
    hipLaunchKernelGGL(k_dots, dim3(nblk, nr), dim3(BS), 0, s, V, ldv, nr, jcount, W, ldw, n, partial, active);
    hipLaunchKernelGGL(k_dots_reduce, dim3(nr), dim3(128), 0, s, partial, nblk, nr, jcount, h, active);
    return hipGetLastError();
}

hipError_t launch_update(const double2* V, size_t ldv, int nr, int jcount, const double2* h, double2* W,
                         size_t ldw, int n, const int* active, double* norm_part, hipStream_t s)
{
    const int nblk = (n + BS - 1) / BS;
    hipLaunchKernelGGL(k_update, dim3(nblk, nr), dim3(BS), 0, s, V, ldv, nr, jcount, h, W, ldw, n, active,
                       norm_part);
    return hipGetLastError();
}

hipError_t launch_arnoldi_finish(int nr, int j, int m, const double2* h1, const double2* h2,
                                 const double* norm_part, int nblk, double2* H, double* hnorm, const int* active,
                                 hipStream_t s)
{
    hipLaunchKernelGGL(k_arnoldi_finish, dim3(nr), dim3(128), 0, s, nr, j, m, h1, h2, norm_part, nblk, H, hnorm,
                       active);
    return hipGetLastError();
}

hipError_t launch_scale_into(const double2* W, size_t ldw, int n, int nr, const double* hnorm, double2* V,
                             size_t ldv, const int* active, hipStream_t s)
{
    hipLaunchKernelGGL(k_scale_into, dim3((n + BS - 1) / BS, nr), dim3(BS), 0, s, W, ldw, n, hnorm, V, ldv, nr,
                       active);
    return hipGetLastError();
}

hipError_t launch_arnoldi_givens(int nr, int j, int m, const double2* h1, const double2* h2,
                                 const double* norm_part, int nblk, double2* H, double2* cs, double2* sn,
                                 double2* gvec, double* hnorm, double* resid, const int* active, hipStream_t s)
{
    hipLaunchKernelGGL(k_arnoldi_givens, dim3(nr), dim3(64), 0, s, nr, j, m, h1, h2, norm_part, nblk, H, cs, sn, gvec,
                       hnorm, resid, active);
    return hipGetLastError();
}

hipError_t launch_givens(int nr, int j, int m, double2* H, double2* cs, double2* sn, double2* gvec, double* resid,
                         const int* active, hipStream_t s)
{
    hipLaunchKernelGGL(k_givens, dim3((nr + 63) / 64), dim3(64), 0, s, nr, j, m, H, cs, sn, gvec, resid, active);
    return hipGetLastError();
}

hipError_t launch_start_cycle(const double2* R, size_t ldr, int n, int nr, const double* rnorm, int m,
                              double2* V, size_t ldv, double2* gvec, const int* active, hipStream_t s)
{
    const int len = std::max(n, m + 1);
    hipLaunchKernelGGL(k_start_cycle, dim3((len + BS - 1) / BS, nr), dim3(BS), 0, s, R, ldr, n, nr, rnorm, m, V,
                       ldv, gvec, active);
    return hipGetLastError();
}

hipError_t launch_backsolve(int nr, int m, const double2* H, const double2* gvec, const int* kdim, double2* y,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_backsolve_wave, dim3(nr), dim3(64), 0, s, nr, m, H, gvec, kdim, y);
    return hipGetLastError();
}

hipError_t launch_xupdate(const double2* V, size_t ldv, int nr, int n, const double2* y, const int* kdim,
                          double2* X, size_t ldx, hipStream_t s)
{
    hipLaunchKernelGGL(k_xupdate, dim3((n + BS - 1) / BS, nr), dim3(BS), 0, s, V, ldv, nr, n, y, kdim, X, ldx);
    return hipGetLastError();
}

hipError_t launch_axpby_res(const double2* B, size_t ldb, const double2* AX, size_t ldax, int n, int nr,
                            double2* R, size_t ldr, hipStream_t s)
{
    hipLaunchKernelGGL(k_axpby_res, dim3((n + BS - 1) / BS, nr), dim3(BS), 0, s, B, ldb, AX, ldax, n, R, ldr);
    return hipGetLastError();
}

hipError_t launch_cast_f64_to_f32(const double2* X, size_t ldx, int n, int nr, float2* Y, size_t ldy, hipStream_t s)
{
    hipLaunchKernelGGL(k_cast_64_32, dim3((n + BS - 1) / BS, nr), dim3(BS), 0, s, X, ldx, n, Y, ldy);
    return hipGetLastError();
}

hipError_t launch_cast_f32_to_f64(const float2* X, size_t ldx, int n, int nr, double2* Y, size_t ldy, hipStream_t s)
{
    hipLaunchKernelGGL(k_cast_32_64, dim3((n + BS - 1) / BS, nr), dim3(BS), 0, s, X, ldx, n, Y, ldy);
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
