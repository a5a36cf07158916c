// matvec.hip -- dense complex products Y = A X of the GMRES solve (Sec. 3.2:
// every Krylov step costs one product with the dense collocation matrix) and
// the residual R = B - A X with FP64 accumulation.
//
// Layouts: A column-major (lda); X, Y column-major blocks, one column per
// right-hand side.  Up to 4 right-hand sides: VALU kernel (k_matvec); more:
// matrix-core kernel (k_matvec_mfma).  Both split the columns over blocks and
// add the split partial sums in a fixed order (k_matvec_reduce).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>

#include "internal.h"
#include "launch.h"

namespace bemk {

int matvec_splits_valu(int n);

namespace {

constexpr int BS = 256;        // threads per block
constexpr int MV_WAVES = 4;    // row tiles per block (64 rows each for VALU, 16 for MFMA)
constexpr int MV_CH = 32;      // X columns staged in LDS per step (VALU kernel)

// ---------------------------------------------------------------------------
// Dense complex product Y = A X, split over columns.  A block holds four waves;
// each wave owns 64 consecutive rows (one row per lane: coalesced 1 KiB loads of
// a column-major A) and the block shares the X values of its column range
// through LDS.  Partial sums of each column split go to `part` and are added
// in split order by k_matvec_reduce.  TA / TX: storage types (double2 or
// float2); ACC: accumulation type.
// ---------------------------------------------------------------------------
template <int NR, class TA, class TX, class ACC>
__global__ __launch_bounds__(BS) void k_matvec(const TA* __restrict__ A, size_t lda, int n,
                                               const TX* __restrict__ X, size_t ldx, int nrhs,
                                               ACC* __restrict__ part, int cps)
{
    using S = decltype(ACC{}.x);
    __shared__ ACC xs[MV_CH][NR];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = (blockIdx.x * MV_WAVES + wave) * 64 + lane;
    const int c0 = blockIdx.y * cps;
    const int c1 = min(n, c0 + cps);
    S ar[NR], ai[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) ar[r] = ai[r] = S(0);
    for (int cb = c0; cb < c1; cb += MV_CH) {
        const int nc = min(MV_CH, c1 - cb);
        __syncthreads();
        for (int t = threadIdx.x; t < MV_CH * NR; t += BS) {
            const int c = t % MV_CH, r = t / MV_CH;
            ACC v;
            v.x = S(0);
            v.y = S(0);
            if (c < nc && r < nrhs) {
                const TX x = X[(size_t)r * ldx + cb + c];
                v.x = (S)x.x;
                v.y = (S)x.y;
            }
            xs[c][r] = v;
        }
        __syncthreads();
        if (row < n) {
            const TA* ap = A + (size_t)cb * lda + row;
            if (nc == MV_CH) {
#pragma unroll 8
                for (int c = 0; c < MV_CH; ++c) {
                    const TA a = ap[(size_t)c * lda];
                    const S axr = (S)a.x, axi = (S)a.y;
#pragma unroll
                    for (int r = 0; r < NR; ++r) {
                        const ACC x = xs[c][r];
                        ar[r] = fma(axr, x.x, ar[r]);
                        ar[r] = fma(-axi, x.y, ar[r]);
                        ai[r] = fma(axr, x.y, ai[r]);
                        ai[r] = fma(axi, x.x, ai[r]);
                    }
                }
            } else {
                for (int c = 0; c < nc; ++c) {
                    const TA a = ap[(size_t)c * lda];
                    const S axr = (S)a.x, axi = (S)a.y;
#pragma unroll
                    for (int r = 0; r < NR; ++r) {
                        const ACC x = xs[c][r];
                        ar[r] = fma(axr, x.x, ar[r]);
                        ar[r] = fma(-axi, x.y, ar[r]);
                        ai[r] = fma(axr, x.y, ai[r]);
                        ai[r] = fma(axi, x.x, ai[r]);
                    }
                }
            }
        }
    }
    if (row < n) {
#pragma unroll
        for (int r = 0; r < NR; ++r)
            if (r < nrhs) {
                ACC v;
                v.x = ar[r];
                v.y = ai[r];
                part[((size_t)blockIdx.y * nrhs + r) * n + row] = v;
            }
    }
}

// Y[:, r] = sum over splits (in order) of the partial products; optionally
// R = B - Y (residual form) when B != nullptr.
template <class ACC, class TY>
__global__ void k_matvec_reduce(const ACC* __restrict__ part, int splits, int n, int nrhs, TY* __restrict__ Y,
                                size_t ldy, const double2* __restrict__ B, size_t ldb)
{
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (row >= n || r >= nrhs) return;
    using S = decltype(ACC{}.x);
    S sr = S(0), si = S(0);
    for (int s = 0; s < splits; ++s) {
        const ACC v = part[((size_t)s * nrhs + r) * n + row];
        sr += v.x;
        si += v.y;
    }
    TY out;
    if (B) {
        const double2 b = B[(size_t)r * ldb + row];
        out.x = (decltype(out.x))(b.x - (double)sr);
        out.y = (decltype(out.y))(b.y - (double)si);
    } else {
        out.x = (decltype(out.x))sr;
        out.y = (decltype(out.y))si;
    }
    Y[(size_t)r * ldy + row] = out;
}


// ---------------------------------------------------------------------------
// Block product on the matrix cores (more than 4 right-hand sides).  The
// complex product is four real products, Yr = Ar Xr + Ai (-Xi), Yi = Ar Xi +
// Ai Xr, each a 16 x 16 x 4 MFMA: one wave owns 16 rows and walks its column
// range 4 columns at a time; lane l holds A[row0 + l % 16][c + l / 16] and
// X[c + l / 16][rhs = l % 16] (X packed right-hand-side fastest, XT[c * 16 + r]),
// and receives result j = 0..3 at row row0 + 4 (l / 16) + j (FP32 MFMA) or
// row0 + (l / 16) + 4 j (FP64 MFMA), right-hand side l % 16 (lane layouts
// checked on gfx950).  No LDS, no broadcast: every lane loads its own operands.
// ---------------------------------------------------------------------------
typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <class T>
struct Mfma;
template <>
struct Mfma<double> {
    using acc = d4v;
    using v2 = double2;
    static __device__ __forceinline__ int out_row(int lk, int j) { return lk + 4 * j; }
    static __device__ __forceinline__ acc run(double a, double b, acc c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <>
struct Mfma<float> {
    using acc = f4v;
    using v2 = float2;
    static __device__ __forceinline__ int out_row(int lk, int j) { return 4 * lk + j; }
    static __device__ __forceinline__ acc run(float a, float b, acc c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

// RT: 16-row tiles per wave (they share each X load); U: column steps in flight;
// G3: complex product with three real products (P1 = Ar Xr, P2 = Ai Xi,
// P3 = (Ar + Ai)(Xr + Xi); Yr = P1 - P2, Yi = P3 - P1 - P2) instead of four.
template <class TA, class T, int RT, int U, bool G3>
__global__ __launch_bounds__(BS) void k_matvec_mfma(const TA* __restrict__ A, size_t lda, int n,
                                                    const typename Mfma<T>::v2* __restrict__ XT, int nrhs,
                                                    typename Mfma<T>::v2* __restrict__ part, int cps)
{
    using M = Mfma<T>;
    using acc = typename M::acc;
    using V2 = typename M::v2;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const int row0 = (blockIdx.x * MV_WAVES + wave) * 16 * RT;
    bool rok[RT];
    const TA* ap[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) {
        const int row = row0 + 16 * t + lr;
        rok[t] = row < n;
        ap[t] = A + (rok[t] ? row : 0);
    }
    const int c0 = blockIdx.y * cps;
    const int c1 = min(n, c0 + cps);
    acc rr0[RT], rr1[RT], ii0[RT], ii1[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) rr0[t] = rr1[t] = ii0[t] = ii1[t] = acc{0, 0, 0, 0};
    int c = c0;
    for (; c + 4 * U <= c1; c += 4 * U) {
        TA a[U][RT];
        V2 x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int col = c + 4 * u + lk;
            x[u] = XT[(size_t)col * 16 + lr];
#pragma unroll
            for (int t = 0; t < RT; ++t) a[u][t] = ap[t][(size_t)col * lda];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                const T ar = rok[t] ? (T)a[u][t].x : T(0), ai = rok[t] ? (T)a[u][t].y : T(0);
                if (G3) {
                    rr0[t] = M::run(ar, x[u].x, rr0[t]);
                    rr1[t] = M::run(ai, x[u].y, rr1[t]);
                    ii0[t] = M::run(ar + ai, x[u].x + x[u].y, ii0[t]);
                } else {
                    rr0[t] = M::run(ar, x[u].x, rr0[t]);
                    rr1[t] = M::run(ai, -x[u].y, rr1[t]);
                    ii0[t] = M::run(ar, x[u].y, ii0[t]);
                    ii1[t] = M::run(ai, x[u].x, ii1[t]);
                }
            }
        }
    }
    for (; c < c1; c += 4) {
        const int col = c + lk;
        const bool ok = col < c1;
        T xr = T(0), xi = T(0);
        if (ok) {
            const V2 x = XT[(size_t)col * 16 + lr];
            xr = x.x;
            xi = x.y;
        }
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            T ar = T(0), ai = T(0);
            if (ok && rok[t]) {
                const TA a = ap[t][(size_t)col * lda];
                ar = (T)a.x;
                ai = (T)a.y;
            }
            if (G3) {
                rr0[t] = M::run(ar, xr, rr0[t]);
                rr1[t] = M::run(ai, xi, rr1[t]);
                ii0[t] = M::run(ar + ai, xr + xi, ii0[t]);
            } else {
                rr0[t] = M::run(ar, xr, rr0[t]);
                rr1[t] = M::run(ai, -xi, rr1[t]);
                ii0[t] = M::run(ar, xi, ii0[t]);
                ii1[t] = M::run(ai, xr, ii1[t]);
            }
        }
    }
    if (lr < nrhs) {
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int r = row0 + 16 * t + M::out_row(lk, j);
                if (r < n) {
                    V2 v;
                    if (G3) {
                        v.x = rr0[t][j] - rr1[t][j];
                        v.y = ii0[t][j] - rr0[t][j] - rr1[t][j];
                    } else {
                        v.x = rr0[t][j] + rr1[t][j];
                        v.y = ii0[t][j] + ii1[t][j];
                    }
                    part[((size_t)blockIdx.y * nrhs + lr) * n + r] = v;
                }
            }
    }
}

// XT[c * 16 + r] = X[r * ldx + c] (r < nr), 0 for nr <= r < 16
template <class TX, class V2>
__global__ void k_pack_xt(const TX* __restrict__ X, size_t ldx, int n, int nr, V2* __restrict__ XT)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = t >> 4, r = t & 15;
    if (c >= n) return;
    V2 v;
    v.x = 0;
    v.y = 0;
    if (r < nr) {
        const TX x = X[(size_t)r * ldx + c];
        v.x = x.x;
        v.y = x.y;
    }
    XT[(size_t)c * 16 + r] = v;
}

// Launch shape of the matrix-core product: row tiles per wave, column steps
// in flight, column splits.  BEM_MV_CFG="rt,u,splits" overrides it (tuning).
struct MfmaCfg {
    int rt, u, splits, g3;
};

MfmaCfg mfma_cfg(int n)
{
    MfmaCfg c{2, 8, 8, 1};
    if (const char* e = getenv("BEM_MV_CFG")) {
        int a = 0, b = 0, d = 0, g = 0;
        const int got = sscanf(e, "%d,%d,%d,%d", &a, &b, &d, &g);
        if (got >= 3 && (a == 1 || a == 2 || a == 4) && (b == 2 || b == 4 || b == 8) && d >= 0 && d <= 64) {
            c = {a, b, d, got == 4 ? (g != 0) : 0};
        }
    }
    if (c.splits == 0) {
        const int rowblocks = (n + 16 * c.rt * MV_WAVES - 1) / (16 * c.rt * MV_WAVES);
        int s = (1024 + rowblocks - 1) / rowblocks;
        s = std::min(s, std::max(1, n / 256));
        c.splits = std::max(1, std::min(s, 64));
    }
    c.splits = std::max(1, std::min(c.splits, std::max(1, n / 64)));
    return c;
}

int mfma_splits(int n) { return mfma_cfg(n).splits; }

template <class TA, class T, class V2>
void launch_mfma_variant(const MfmaCfg& c, dim3 grid, hipStream_t s, const TA* A, size_t lda, int n, const V2* xt,
                         int nr, V2* part, int cps)
{
#define BEM_MV_CASE(RT_, U_)                                                                                   \
    if (c.rt == RT_ && c.u == U_) {                                                                            \
        if (c.g3)                                                                                              \
            hipLaunchKernelGGL((k_matvec_mfma<TA, T, RT_, U_, true>), grid, dim3(BS), 0, s, A, lda, n, xt, nr, part, \
                               cps);                                                                           \
        else                                                                                                   \
            hipLaunchKernelGGL((k_matvec_mfma<TA, T, RT_, U_, false>), grid, dim3(BS), 0, s, A, lda, n, xt, nr,    \
                               part, cps);                                                                     \
        return;                                                                                                \
    }
    BEM_MV_CASE(1, 2)
    BEM_MV_CASE(1, 4)
    BEM_MV_CASE(1, 8)
    BEM_MV_CASE(2, 2)
    BEM_MV_CASE(2, 4)
    BEM_MV_CASE(2, 8)
    BEM_MV_CASE(4, 2)
    BEM_MV_CASE(4, 4)
    BEM_MV_CASE(4, 8)
#undef BEM_MV_CASE
}

template <class TA, class TX, class ACC, class TY>
hipError_t matvec_any(const TA* A, size_t lda, int n, const TX* X, size_t ldx, int nrhs, TY* Y, size_t ldy,
                      ACC* part, const double2* B, size_t ldb, hipStream_t s, const KernelHook* hook)
{
    const int splits = matvec_splits_valu(n);
    const int cps = (n + splits - 1) / splits;
    const int rowblocks = (n + 64 * MV_WAVES - 1) / (64 * MV_WAVES);
    using S = decltype(ACC{}.x);
    for (int r0 = 0; r0 < nrhs; r0 += 16) {
        const int nr = std::min(16, nrhs - r0);
        dim3 grid(rowblocks, splits);
        const TX* Xg = X + (size_t)r0 * ldx;
        if (nr > 4) {
            // pack X right-hand-side fastest into the tail of the partial buffer
            const MfmaCfg cfg = mfma_cfg(n);
            const int ms = cfg.splits;
            const int mcps = ((n + ms - 1) / ms + 31) / 32 * 32;
            ACC* xt = part + (size_t)ms * nr * n;
            hipLaunchKernelGGL((k_pack_xt<TX, ACC>), dim3((n * 16 + BS - 1) / BS), dim3(BS), 0, s, Xg, ldx, n, nr, xt);
            hook_call(hook, KIND_MATVEC, 0, s);
            const int rows_per_block = 16 * cfg.rt * MV_WAVES;
            launch_mfma_variant<TA, S, ACC>(cfg, dim3((n + rows_per_block - 1) / rows_per_block, ms), s, A, lda, n, xt,
                                            nr, part, mcps);
            hook_call(hook, KIND_MATVEC, 1, s);
            hipLaunchKernelGGL((k_matvec_reduce<ACC, TY>), dim3((n + BS - 1) / BS, nr), dim3(BS), 0, s, part, ms, n,
                               nr, Y + (size_t)r0 * ldy, ldy, B ? B + (size_t)r0 * ldb : nullptr, ldb);
            continue;
        }
        hook_call(hook, KIND_MATVEC, 0, s);
        if (nr == 1)
            hipLaunchKernelGGL((k_matvec<1, TA, TX, ACC>), grid, dim3(BS), 0, s, A, lda, n, Xg, ldx, nr, part, cps);
        else if (nr == 2)
            hipLaunchKernelGGL((k_matvec<2, TA, TX, ACC>), grid, dim3(BS), 0, s, A, lda, n, Xg, ldx, nr, part, cps);
        else if (nr <= 4)
            hipLaunchKernelGGL((k_matvec<4, TA, TX, ACC>), grid, dim3(BS), 0, s, A, lda, n, Xg, ldx, nr, part, cps);
        else if (nr <= 8)
            hipLaunchKernelGGL((k_matvec<8, TA, TX, ACC>), grid, dim3(BS), 0, s, A, lda, n, Xg, ldx, nr, part, cps);
        else
            hipLaunchKernelGGL((k_matvec<16, TA, TX, ACC>), grid, dim3(BS), 0, s, A, lda, n, Xg, ldx, nr, part,
                               cps);
        hook_call(hook, KIND_MATVEC, 1, s);
        hipLaunchKernelGGL((k_matvec_reduce<ACC, TY>), dim3((n + BS - 1) / BS, nr), dim3(BS), 0, s, part, splits, n,
                           nr, Y + (size_t)r0 * ldy, ldy, B ? B + (size_t)r0 * ldb : nullptr, ldb);
    }
    return hipGetLastError();
}

}  // namespace

int matvec_splits_valu(int n)
{
    // enough column splits that the grid holds >= ~1024 blocks of 4 waves,
    // but never fewer than 64 columns per split
    const int rowblocks = (n + 64 * MV_WAVES - 1) / (64 * MV_WAVES);
    int s = (1024 + rowblocks - 1) / rowblocks;
    const int maxs = std::max(1, n / 64);
    if (s > maxs) s = maxs;
    if (s > 64) s = 64;
    return std::max(1, s);
}

// partial-sum buffer in units of n complex values: the largest split count any
// launch shape may use plus the packed copy of X (16 columns)
int matvec_splits(int n) { return std::max(matvec_splits_valu(n), 64 + 16); }

hipError_t launch_matvec_f64(const double2* A, size_t lda, int n, const double2* X, size_t ldx, int nrhs,
                             double2* Y, size_t ldy, double2* partial, hipStream_t s, const KernelHook* hook)
{
    return matvec_any<double2, double2, double2, double2>(A, lda, n, X, ldx, nrhs, Y, ldy, partial, nullptr, 0, s,
                                                          hook);
}

hipError_t launch_matvec_f32(const float2* A, size_t lda, int n, const float2* X, size_t ldx, int nrhs, float2* Y,
                             size_t ldy, float2* partial, hipStream_t s, const KernelHook* hook)
{
    return matvec_any<float2, float2, float2, float2>(A, lda, n, X, ldx, nrhs, Y, ldy, partial, nullptr, 0, s, hook);
}

hipError_t launch_residual_f64(const double2* A, size_t lda, int n, const double2* X, size_t ldx, int nrhs,
                              const double2* B, size_t ldb, double2* R, size_t ldr, double2* partial, hipStream_t s,
                              const KernelHook* hook)
{
    return matvec_any<double2, double2, double2, double2>(A, lda, n, X, ldx, nrhs, R, ldr, partial, B, ldb, s, hook);
}

hipError_t launch_residual_f32A(const float2* A, size_t lda, int n, const double2* X, size_t ldx, int nrhs,
                                const double2* B, size_t ldb, double2* R, size_t ldr, double2* partial,
                                hipStream_t s, const KernelHook* hook)
{
    return matvec_any<float2, double2, double2, double2>(A, lda, n, X, ldx, nrhs, R, ldr, partial, B, ldb, s, hook);
}

}  // namespace bemk
