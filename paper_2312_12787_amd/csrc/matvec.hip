// matvec.hip -- dense complex products Y = A X of the GMRES solve (Sec. 3.2:
// every Krylov step costs one product with the dense collocation matrix) and
// the residual R = B - A X with FP64 accumulation.
//
// Layouts: A column-major (lda); X, Y column-major blocks, one column per
// right-hand side.  Up to 4 right-hand sides: VALU kernel (k_matvec); more:
// matrix-core kernel (k_matvec_mfma), up to 64 right-hand sides per pass over A.  Both split the columns over blocks and
// add the split partial sums in a fixed order (k_matvec_reduce).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "internal.h"
#include "krylov_dev.h"
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
// The matrix is streamed once per product and is larger than the caches:
// non-temporal loads keep it from displacing the reused X blocks (measured on
// gfx950: 2.7 % faster FP64 products at n = 8192, 16 right-hand sides).
template <class TA>
__device__ __forceinline__ TA ld_stream(const TA* p)
{
    TA v;
    v.x = __builtin_nontemporal_load(&p->x);
    v.y = __builtin_nontemporal_load(&p->y);
    return v;
}

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
                    const TA a = ld_stream(ap + (size_t)c * lda);
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
                    const TA a = ld_stream(ap + (size_t)c * lda);
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
// P3 = (Ar + Ai)(Xr + Xi); Yr = P1 - P2, Yi = P3 - P1 - P2) instead of four;
// NG: groups of 16 right-hand sides taken in the same pass over A (X packed
// XT[c * 16 NG + r]), so that one read of A serves up to 64 right-hand sides.
// The wide shapes, which are matrix-core bound, carry an occupancy target:
// left alone the compiler puts their accumulators in AGPRs beside the load
// slots and runs one or two waves per SIMD; with the target they fit in the
// VGPRs without spilling (FP32 sums with 64 right-hand sides: three waves,
// 3.49 -> 3.45 ms per kite16384 product; FP64 sums over two to four groups,
// where RT * NG <= 4 keeps them spill-free: two waves, the kite16384 FP64
// path 73.7 -> 84.4 solves/s).  The single-group shapes keep the compiler's
// own allocation (the HBM-bound 16-RHS product pipelines its loads instead).
constexpr int mfma_min_waves(int tbytes, int rt, int ng)
{
    return (tbytes == 4 && ng >= 4) ? 3 : (tbytes == 8 && ng >= 2 && rt * ng <= 4) ? 2 : 1;
}

template <class TA, class T, int RT, int U, bool G3, int NG>
__global__ __launch_bounds__(BS, mfma_min_waves(sizeof(T), RT, NG)) void k_matvec_mfma(const TA* __restrict__ A, size_t lda, int n,
                                                    const typename Mfma<T>::v2* __restrict__ XT, int nrhs,
                                                    typename Mfma<T>::v2* __restrict__ part, int cps)
{
    using M = Mfma<T>;
    using acc = typename M::acc;
    using V2 = typename M::v2;
    constexpr int XW = 16 * NG;
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
    acc rr0[NG][RT], rr1[NG][RT], ii0[NG][RT], ii1[NG][RT];
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
        for (int t = 0; t < RT; ++t) rr0[g][t] = rr1[g][t] = ii0[g][t] = ii1[g][t] = acc{0, 0, 0, 0};
    // one 16 x 4 tile of A (per row tile) against 4 x 16 NG of X
    auto step = [&](const T (&ar)[RT], const T (&ai)[RT], const T (&xr)[NG], const T (&xi)[NG]) {
#pragma unroll
        for (int g = 0; g < NG; ++g)
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                if (G3) {
                    rr0[g][t] = M::run(ar[t], xr[g], rr0[g][t]);
                    rr1[g][t] = M::run(ai[t], xi[g], rr1[g][t]);
                    ii0[g][t] = M::run(ar[t] + ai[t], xr[g] + xi[g], ii0[g][t]);
                } else {
                    rr0[g][t] = M::run(ar[t], xr[g], rr0[g][t]);
                    rr1[g][t] = M::run(ai[t], -xi[g], rr1[g][t]);
                    ii0[g][t] = M::run(ar[t], xi[g], ii0[g][t]);
                    ii1[g][t] = M::run(ai[t], xr[g], ii1[g][t]);
                }
            }
    };
    // HBM-bound shapes (one group of 16 right-hand sides, at most 16 tile
    // loads per step) walk the columns software-pipelined: the loads of the
    // next 4U columns are issued before the products of the current ones, so
    // a wave keeps its reads in flight while its matrix-core work runs.  The
    // wider shapes, matrix-core bound, would spill a second buffer; they
    // rotate their slots instead (below).
    constexpr bool PIPE = NG == 1 && RT * U <= 16;
    auto load = [&](TA (&a)[U][RT], V2 (&x)[U][NG], int cc) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int col = cc + 4 * u + lk;
#pragma unroll
            for (int g = 0; g < NG; ++g) x[u][g] = XT[(size_t)col * XW + 16 * g + lr];
#pragma unroll
            for (int t = 0; t < RT; ++t) a[u][t] = ld_stream(ap[t] + (size_t)col * lda);
        }
    };
    auto compute = [&](const TA (&a)[U][RT], const V2 (&x)[U][NG]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            T ar[RT], ai[RT], xr[NG], xi[NG];
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                ar[t] = rok[t] ? (T)a[u][t].x : T(0);
                ai[t] = rok[t] ? (T)a[u][t].y : T(0);
            }
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                xr[g] = x[u][g].x;
                xi[g] = x[u][g].y;
            }
            step(ar, ai, xr, xi);
        }
    };
    int c = c0;
    if constexpr (!PIPE) {
        // rotating slots: slot u of the next 4U columns is loaded as soon as
        // slot u of the current ones has gone into the matrix cores, so a
        // wave keeps loads in flight without a second buffer; the scheduling
        // barriers keep that order (the compiler otherwise moves the loads
        // next to their uses and waits for all of them).  Measured on gfx950,
        // kite of 16384 elements, 64 right-hand sides: FP32 product 3.82 ->
        // 3.50 ms at the same register count (two waves per SIMD)
        if (c + 4 * U <= c1) {
            TA a[U][RT];
            V2 x[U][NG];
            load(a, x, c);
            for (;;) {
                const int cn = c + 4 * U;
                const bool more = cn + 4 * U <= c1;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    T ar[RT], ai[RT], xr[NG], xi[NG];
#pragma unroll
                    for (int t = 0; t < RT; ++t) {
                        ar[t] = rok[t] ? (T)a[u][t].x : T(0);
                        ai[t] = rok[t] ? (T)a[u][t].y : T(0);
                    }
#pragma unroll
                    for (int g = 0; g < NG; ++g) {
                        xr[g] = x[u][g].x;
                        xi[g] = x[u][g].y;
                    }
                    step(ar, ai, xr, xi);
                    __builtin_amdgcn_sched_barrier(0);
                    // unconditional (the last pass reloads its own columns):
                    // a load under a branch makes the compiler wait for every
                    // load in flight before the next slot
                    const int col = (more ? cn : c) + 4 * u + lk;
#pragma unroll
                    for (int g = 0; g < NG; ++g) x[u][g] = XT[(size_t)col * XW + 16 * g + lr];
#pragma unroll
                    for (int t = 0; t < RT; ++t) a[u][t] = ld_stream(ap[t] + (size_t)col * lda);
                    __builtin_amdgcn_sched_barrier(0);
                }
                c = cn;
                if (!more) break;
            }
        }
    } else if (c + 4 * U <= c1) {
        TA a[U][RT];
        V2 x[U][NG];
        load(a, x, c);
        for (;;) {
            const int cn = c + 4 * U;
            if (cn + 4 * U > c1) {
                compute(a, x);
                c = cn;
                break;
            }
            TA an[U][RT];
            V2 xn[U][NG];
            load(an, xn, cn);
            compute(a, x);
#pragma unroll
            for (int u = 0; u < U; ++u) {
#pragma unroll
                for (int t = 0; t < RT; ++t) a[u][t] = an[u][t];
#pragma unroll
                for (int g = 0; g < NG; ++g) x[u][g] = xn[u][g];
            }
            c = cn;
        }
    }
    for (; c < c1; c += 4) {
        const int col = c + lk;
        const bool ok = col < c1;
        T ar[RT], ai[RT], xr[NG], xi[NG];
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            xr[g] = T(0);
            xi[g] = T(0);
            if (ok) {
                const V2 x = XT[(size_t)col * XW + 16 * g + lr];
                xr[g] = x.x;
                xi[g] = x.y;
            }
        }
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            ar[t] = T(0);
            ai[t] = T(0);
            if (ok && rok[t]) {
                const TA a = ld_stream(ap[t] + (size_t)col * lda);
                ar[t] = (T)a.x;
                ai[t] = (T)a.y;
            }
        }
        step(ar, ai, xr, xi);
    }
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        const int r = 16 * g + lr;
        if (r >= nrhs) continue;
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int row = row0 + 16 * t + M::out_row(lk, j);
                if (row < n) {
                    V2 v;
                    if (G3) {
                        v.x = rr0[g][t][j] - rr1[g][t][j];
                        v.y = ii0[g][t][j] - rr0[g][t][j] - rr1[g][t][j];
                    } else {
                        v.x = rr0[g][t][j] + rr1[g][t][j];
                        v.y = ii0[g][t][j] + ii1[g][t][j];
                    }
                    part[((size_t)blockIdx.y * nrhs + r) * n + row] = v;
                }
            }
    }
}

// XT[c * xw + r] = X[r * ldx + c] (r < nr), 0 for nr <= r < xw (xw = 16, 32, 48, 64)
template <class TX, class V2>
__global__ void k_pack_xt(const TX* __restrict__ X, size_t ldx, int n, int nr, int xw, V2* __restrict__ XT)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = t / xw, r = t - c * xw;
    if (c >= n) return;
    V2 v;
    v.x = 0;
    v.y = 0;
    if (r < nr) {
        const TX x = X[(size_t)r * ldx + c];
        v.x = x.x;
        v.y = x.y;
    }
    XT[(size_t)c * xw + r] = v;
}

// Launch shape of the matrix-core product: row tiles per wave, column steps
// in flight, column splits (0: enough for about 1024 blocks), 3-product form,
// for one group of 16 right-hand sides and for 2-4 groups per pass.
MvShape mfma_default(int n, int ng, bool f64)
{
    // defaults measured on gfx950 (n = 32768; 16, 32 and 64 right-hand sides;
    // FP64 sums over 3-4 groups take one row tile, which runs two waves per
    // SIMD: the mixed path's 64-RHS refinement residual 7.73 -> 6.29 ms)
    MvShape c = ng == 1 ? MvShape{2, 8, 8, 1} : (f64 && ng == 2 ? MvShape{1, 4, 8, 1} : MvShape{f64 ? 1 : 2, 4, 0, 1});
    if (c.splits == 0) {
        const int rowblocks = (n + 16 * c.rt * MV_WAVES - 1) / (16 * c.rt * MV_WAVES);
        int s = (1024 + rowblocks - 1) / rowblocks;
        s = std::min(s, std::max(1, n / 256));
        c.splits = std::max(1, std::min(s, 64));
    }
    c.splits = std::max(1, std::min(c.splits, std::max(1, n / 64)));
    return c;
}

bool shape_valid(int ng, const MvShape& c)
{
    if (ng == 0) return c.splits >= 1 && c.splits <= 64;
    const bool ok = ng == 1 ? ((c.rt == 1 || c.rt == 2 || c.rt == 4) && (c.u == 2 || c.u == 4 || c.u == 8))
                            : ((c.rt == 1 || c.rt == 2) && (c.u == 2 || c.u == 4) && c.g3 == 1);
    return ok && c.splits >= 1 && c.splits <= 64;
}

// ---------------------------------------------------------------------------
// Launch-shape table.  A class is (type pair, right-hand-side groups, size
// class): types = 2 [matrix stored in FP64] + [accumulation in FP64]; ng = 0
// for the vector kernel (up to 4 right-hand sides), 1-4 for the matrix-core
// kernel; size class = ceil(log2 n).  bem_tune fills the table; the tuner's
// candidate under test is forced per thread.  Column splits never exceed
// split_cap(n, ng), by which the partial-sum buffer is sized, so buffers sized
// before or after tuning stay valid.
// ---------------------------------------------------------------------------
struct ShapeKey {
    int types, ng, lg;
    bool operator<(const ShapeKey& o) const
    {
        return types != o.types ? types < o.types : (ng != o.ng ? ng < o.ng : lg < o.lg);
    }
};
std::mutex g_tune_mu;
std::map<ShapeKey, MvShape> g_tuned;
thread_local const MvShape* g_forced = nullptr;

int size_class(int n)
{
    int lg = 0;
    while (lg < 31 && (1 << lg) < n) ++lg;
    return lg;
}

int split_cap(int n, int ng)
{
    if (ng == 0) return matvec_splits_valu(n);
    const int want = (131072 + n - 1) / std::max(1, n);  // about 2048 blocks at one row tile per wave
    const int cap = std::max(1, std::min({want, 64, std::max(1, n / 64)}));
    return std::max(cap, std::max(mfma_default(n, ng, true).splits, mfma_default(n, ng, false).splits));
}

// Environment overrides of the launch shape (manual tuning): BEM_MV_CFG for
// one group of 16 right-hand sides, BEM_MV_CFG_WIDE for 2-4 groups,
// "rt,u,splits[,g3]".
bool env_shape(int ng, MvShape& out)
{
    const char* e = getenv(ng == 1 ? "BEM_MV_CFG" : "BEM_MV_CFG_WIDE");
    if (!e) return false;
    MvShape t{0, 0, 0, 1};
    const int got = sscanf(e, "%d,%d,%d,%d", &t.rt, &t.u, &t.splits, &t.g3);
    if (ng > 1) t.g3 = 1;
    t.g3 = t.g3 != 0;
    if (got < 3 || !shape_valid(ng, t)) return false;
    out = t;
    return true;
}

}  // namespace

// A frozen source of shapes: the tuned table and the environment overrides.
struct ShapeSnapshot {
    std::map<ShapeKey, MvShape> table;
    bool have_env[2] = {false, false};  // [0]: one group, [1]: 2-4 groups
    MvShape env[2] = {};
};

namespace {

// The shape a product of this class runs with, from a snapshot (or the live
// table and environment when snap is null): an environment override, else the
// tuned table, else the default; splits clamped to split_cap.
MvShape shape_from(const ShapeSnapshot* snap, int types, int ng, int n)
{
    MvShape c = ng == 0 ? MvShape{0, 0, matvec_splits_valu(n), 0} : mfma_default(n, ng, types & 1);
    bool have = false;
    if (ng > 0) {
        MvShape t{};
        if (snap ? snap->have_env[ng > 1] : env_shape(ng, t)) {
            c = snap ? snap->env[ng > 1] : t;
            have = true;
        }
    }
    if (!have) {
        const ShapeKey key{types, ng, size_class(n)};
        if (snap) {
            auto it = snap->table.find(key);
            if (it != snap->table.end()) c = it->second;
        } else {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tuned.find(key);
            if (it != g_tuned.end()) c = it->second;
        }
    }
    c.splits = std::max(1, std::min({c.splits, split_cap(n, ng), std::max(1, n / 64)}));
    return c;
}

// The shape a launch uses: the tuner's forced candidate (this thread), else the
// problem's resolved shapes, else the live table (callers without a problem).
MvShape pick_shape(const MvShapes* shapes, int types, int ng, int n)
{
    if (g_forced && shape_valid(ng, *g_forced)) {
        MvShape c = *g_forced;
        c.splits = std::max(1, std::min({c.splits, split_cap(n, ng), std::max(1, n / 64)}));
        return c;
    }
    if (shapes) return shapes->s[types][ng];
    return shape_from(nullptr, types, ng, n);
}

constexpr int MFMA_MAX_RHS = 64;  // right-hand sides per pass over A

template <class TA, class T, class V2>
void launch_mfma_variant(const MvShape& c, int ng, dim3 grid, hipStream_t s, const TA* A, size_t lda, int n,
                         const V2* xt, int nr, V2* part, int cps)
{
#define BEM_MV_LAUNCH(RT_, U_, G3_, NG_) \
    hipLaunchKernelGGL((k_matvec_mfma<TA, T, RT_, U_, G3_, NG_>), grid, dim3(BS), 0, s, A, lda, n, xt, nr, part, cps)
#define BEM_MV_CASE(RT_, U_)                         \
    if (c.rt == RT_ && c.u == U_) {                  \
        if (c.g3)                                    \
            BEM_MV_LAUNCH(RT_, U_, true, 1);         \
        else                                         \
            BEM_MV_LAUNCH(RT_, U_, false, 1);        \
        return;                                      \
    }
#define BEM_MV_WIDE(RT_, U_)                                  \
    if (c.rt == RT_ && c.u == U_) {                           \
        if (ng == 2)                                          \
            BEM_MV_LAUNCH(RT_, U_, true, 2);                  \
        else if (ng == 3)                                     \
            BEM_MV_LAUNCH(RT_, U_, true, 3);                  \
        else                                                  \
            BEM_MV_LAUNCH(RT_, U_, true, 4);                  \
        return;                                               \
    }
    if (ng == 1) {
        BEM_MV_CASE(1, 2)
        BEM_MV_CASE(1, 4)
        BEM_MV_CASE(1, 8)
        BEM_MV_CASE(2, 2)
        BEM_MV_CASE(2, 4)
        BEM_MV_CASE(2, 8)
        BEM_MV_CASE(4, 2)
        BEM_MV_CASE(4, 4)
        BEM_MV_CASE(4, 8)
    } else {
        BEM_MV_WIDE(1, 2)
        BEM_MV_WIDE(1, 4)
        BEM_MV_WIDE(2, 2)
        BEM_MV_WIDE(2, 4)
    }
#undef BEM_MV_WIDE
#undef BEM_MV_CASE
#undef BEM_MV_LAUNCH
}

template <class TA, class TX, class ACC, class TY>
hipError_t matvec_any(const TA* A, size_t lda, int n, const TX* X, size_t ldx, int nrhs, TY* Y, size_t ldy,
                      ACC* part, const double2* B, size_t ldb, hipStream_t s, const KernelHook* hook,
                      const MvShapes* shapes)
{
    using S = decltype(ACC{}.x);
    constexpr int types = (sizeof(TA) == 16 ? 2 : 0) + (sizeof(S) == 8 ? 1 : 0);
    const int splits = pick_shape(shapes, types, 0, n).splits;
    const int cps = (n + splits - 1) / splits;
    const int rowblocks = (n + 64 * MV_WAVES - 1) / (64 * MV_WAVES);
    const int kind = B ? KIND_RESIDUAL : KIND_MATVEC;
    for (int r0 = 0; r0 < nrhs; r0 += MFMA_MAX_RHS) {
        const int nr = std::min(MFMA_MAX_RHS, nrhs - r0);
        const TX* Xg = X + (size_t)r0 * ldx;
        if (nr > 4) {
            // pack X right-hand-side fastest into the tail of the partial buffer
            const int ng = (nr + 15) / 16;
            const MvShape cfg = pick_shape(shapes, types, ng, n);
            const int ms = cfg.splits;
            const int mcps = ((n + ms - 1) / ms + 31) / 32 * 32;
            ACC* xt = part + (size_t)ms * nr * n;
            hipLaunchKernelGGL((k_pack_xt<TX, ACC>), dim3(((size_t)n * 16 * ng + BS - 1) / BS), dim3(BS), 0, s, Xg,
                               ldx, n, nr, 16 * ng, xt);
            hook_call(hook, kind, 0, s);
            const int rows_per_block = 16 * cfg.rt * MV_WAVES;
            launch_mfma_variant<TA, S, ACC>(cfg, ng, dim3((n + rows_per_block - 1) / rows_per_block, ms), s, A, lda,
                                            n, xt, nr, part, mcps);
            hook_call(hook, kind, 1, s);
            hipLaunchKernelGGL((k_matvec_reduce<ACC, TY>), dim3((n + BS - 1) / BS, nr), dim3(BS), 0, s, part, ms, n,
                               nr, Y + (size_t)r0 * ldy, ldy, B ? B + (size_t)r0 * ldb : nullptr, ldb);
            continue;
        }
        dim3 grid(rowblocks, splits);
        hook_call(hook, kind, 0, s);
        if (nr == 1)
            hipLaunchKernelGGL((k_matvec<1, TA, TX, ACC>), grid, dim3(BS), 0, s, A, lda, n, Xg, ldx, nr, part, cps);
        else if (nr == 2)
            hipLaunchKernelGGL((k_matvec<2, TA, TX, ACC>), grid, dim3(BS), 0, s, A, lda, n, Xg, ldx, nr, part, cps);
        else
            hipLaunchKernelGGL((k_matvec<4, TA, TX, ACC>), grid, dim3(BS), 0, s, A, lda, n, Xg, ldx, nr, part, cps);
        hook_call(hook, kind, 1, s);
        hipLaunchKernelGGL((k_matvec_reduce<ACC, TY>), dim3((n + BS - 1) / BS, nr), dim3(BS), 0, s, part, splits, n,
                           nr, Y + (size_t)r0 * ldy, ldy, B ? B + (size_t)r0 * ldb : nullptr, ldb);
    }
    return hipGetLastError();
}

__device__ __forceinline__ void st_basis(double2* p, double2 v) { *p = v; }
__device__ __forceinline__ void st_basis(float2* p, double2 v) { *p = make_float2((float)v.x, (float)v.y); }

// The split reduction of a Krylov step's product whose inputs were w of the
// previous step, not yet divided by |w|: Y = (sum of the split partial sums,
// in split order) / |w| = A v_j, and before Y overwrites w (Y is the step's w
// buffer): v_j = w / |w| into the basis for active columns, |w| into hnorm,
// and the stopping marks of the previous step cleared (what the
// normalisation kernel does otherwise).
template <class ACC, class TV>
__global__ void k_step_reduce(const ACC* __restrict__ part, int splits, int n, int nrhs, double2* __restrict__ Y,
                              size_t ldy, const double* __restrict__ nrm, int nu, TV* __restrict__ V, size_t ldv,
                              double* __restrict__ hnorm, int* __restrict__ active)
{
    __shared__ double inv_s;
    const int r = blockIdx.y;
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    const int act = active[r];
    // this thread's loads first (they do not depend on |w|), then |w|
    using S = decltype(ACC{}.x);
    S sr = S(0), si = S(0);
    double2 w = make_double2(0.0, 0.0);
    double2* y = Y + (size_t)r * ldy + row;
    if (row < n) {
        for (int sp = 0; sp < splits; ++sp) {
            const ACC v = part[((size_t)sp * nrhs + r) * n + row];
            sr += v.x;
            si += v.y;
        }
        w = *y;
    }
    if (threadIdx.x < 64) {
        const double beta = dev::step_beta(nrm + (size_t)r * nu, nu);
        if (threadIdx.x == 0) {
            inv_s = dev::inv_beta(beta);
            if (blockIdx.x == 0 && act == 1) hnorm[r] = beta;
        }
    }
    __syncthreads();
    // every block of a marked column skips it, whether it reads the mark or the zero
    if (blockIdx.x == 0 && threadIdx.x == 0 && act == dev::STOPPING) active[r] = 0;
    if (row >= n) return;
    const double inv = inv_s;
    if (act == 1) st_basis(V + (size_t)r * ldv + row, make_double2(w.x * inv, w.y * inv));
    *y = make_double2((double)sr * inv, (double)si * inv);
}

// Products of the Krylov steps with 5-64 right-hand sides, packed by the
// caller at part + xt_offset: the matrix-core kernel and the split reduction
// (with sn: inputs not yet normalised, see k_step_reduce).
template <class TA, class ACC>
hipError_t product_packed(const ProductPlan& pl, const TA* A, size_t lda, int n, int nr, ACC* part, double2* Y,
                          size_t ldy, const StepNorm* sn, hipStream_t s, const KernelHook* hook)
{
    using S = decltype(ACC{}.x);
    const int rows_per_block = 16 * pl.shape.rt * MV_WAVES;
    const int mcps = ((n + pl.splits - 1) / pl.splits + 31) / 32 * 32;
    hook_call(hook, KIND_MATVEC, 0, s);
    launch_mfma_variant<TA, S, ACC>(pl.shape, pl.ng, dim3((n + rows_per_block - 1) / rows_per_block, pl.splits), s, A,
                                    lda, n, part + pl.xt_offset, nr, part, mcps);
    hook_call(hook, KIND_MATVEC, 1, s);
    const dim3 grid((n + BS - 1) / BS, nr);
    if (!sn)
        hipLaunchKernelGGL((k_matvec_reduce<ACC, double2>), grid, dim3(BS), 0, s, part, pl.splits, n, nr, Y, ldy,
                           nullptr, 0);
    else if (sn->v32)
        hipLaunchKernelGGL((k_step_reduce<ACC, float2>), grid, dim3(BS), 0, s, part, pl.splits, n, nr, Y, ldy,
                           sn->norm_part, sn->nu, static_cast<float2*>(sn->V), sn->ldv, sn->hnorm, sn->active);
    else
        hipLaunchKernelGGL((k_step_reduce<ACC, double2>), grid, dim3(BS), 0, s, part, pl.splits, n, nr, Y, ldy,
                           sn->norm_part, sn->nu, static_cast<double2*>(sn->V), sn->ldv, sn->hnorm, sn->active);
    return hipGetLastError();
}

}  // namespace

ProductPlan product_plan(const MvShapes* shapes, int types, int n, int nr)
{
    ProductPlan pl{};
    pl.ng = nr > 4 ? (nr + 15) / 16 : 0;
    pl.shape = pick_shape(shapes, types, pl.ng, n);
    pl.splits = pl.shape.splits;
    pl.xt_offset = pl.ng > 0 ? (size_t)pl.splits * nr * n : 0;
    pl.xw = 16 * pl.ng;
    return pl;
}

hipError_t launch_product_packed_f64(const ProductPlan& pl, const double2* A, size_t lda, int n, int nr,
                                     double2* part, double2* Y, size_t ldy, const StepNorm* sn, hipStream_t s,
                                     const KernelHook* hook)
{
    return product_packed<double2, double2>(pl, A, lda, n, nr, part, Y, ldy, sn, s, hook);
}

hipError_t launch_product_packed_f32(const ProductPlan& pl, const float2* A, size_t lda, int n, int nr,
                                     float2* part, double2* Y, size_t ldy, const StepNorm* sn, hipStream_t s,
                                     const KernelHook* hook)
{
    return product_packed<float2, float2>(pl, A, lda, n, nr, part, Y, ldy, sn, s, hook);
}

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

// Partial-sum buffer of a product with nrhs right-hand sides, in complex
// values of the accumulation type: the column-split partial sums of the
// largest chunk plus the packed copy of X (matrix-core path).  Sized for the
// FP64 shape; an FP32 product uses the same shape with half-size values.
size_t matvec_part_elems(int n, int nrhs)
{
    const int nr = std::min(nrhs, MFMA_MAX_RHS);
    size_t e = (size_t)split_cap(n, 0) * std::min(nr, 4);
    if (nr > 4) {
        const int ng = (nr + 15) / 16;
        e = std::max(e, (size_t)split_cap(n, ng) * nr + 16 * ng);
    }
    return e * (size_t)n;
}

size_t matvec_part_elems_shaped(const MvShapes& sh, int types, int n, int nrhs)
{
    size_t e = 0;
    for (int r0 = 0; r0 < nrhs; r0 += MFMA_MAX_RHS) {
        const int nr = std::min(MFMA_MAX_RHS, nrhs - r0);
        const int ng = nr > 4 ? (nr + 15) / 16 : 0;
        const size_t c = (size_t)sh.s[types][ng].splits * nr + (ng ? 16 * ng : 0);
        e = std::max(e, c);
    }
    return e * (size_t)n;
}

hipError_t launch_matvec_f64(const double2* A, size_t lda, int n, const double2* X, size_t ldx, int nrhs,
                             double2* Y, size_t ldy, double2* partial, hipStream_t s, const KernelHook* hook,
                             const MvShapes* shapes)
{
    return matvec_any<double2, double2, double2, double2>(A, lda, n, X, ldx, nrhs, Y, ldy, partial, nullptr, 0, s,
                                                          hook, shapes);
}

hipError_t launch_matvec_f32(const float2* A, size_t lda, int n, const float2* X, size_t ldx, int nrhs, float2* Y,
                             size_t ldy, float2* partial, hipStream_t s, const KernelHook* hook,
                             const MvShapes* shapes)
{
    return matvec_any<float2, float2, float2, float2>(A, lda, n, X, ldx, nrhs, Y, ldy, partial, nullptr, 0, s, hook,
                                                      shapes);
}

hipError_t launch_matvec_f32x64(const float2* A, size_t lda, int n, const double2* X, size_t ldx, int nrhs,
                                double2* Y, size_t ldy, float2* partial, hipStream_t s, const KernelHook* hook,
                             const MvShapes* shapes)
{
    return matvec_any<float2, double2, float2, double2>(A, lda, n, X, ldx, nrhs, Y, ldy, partial, nullptr, 0, s, hook,
                                                        shapes);
}

hipError_t launch_matvec_f32v(const float2* A, size_t lda, int n, const float2* X, size_t ldx, int nrhs,
                              double2* Y, size_t ldy, float2* partial, hipStream_t s, const KernelHook* hook,
                             const MvShapes* shapes)
{
    return matvec_any<float2, float2, float2, double2>(A, lda, n, X, ldx, nrhs, Y, ldy, partial, nullptr, 0, s, hook,
                                                       shapes);
}

hipError_t launch_residual_f64(const double2* A, size_t lda, int n, const double2* X, size_t ldx, int nrhs,
                              const double2* B, size_t ldb, double2* R, size_t ldr, double2* partial, hipStream_t s,
                              const KernelHook* hook, const MvShapes* shapes)
{
    return matvec_any<double2, double2, double2, double2>(A, lda, n, X, ldx, nrhs, R, ldr, partial, B, ldb, s, hook,
                                                          shapes);
}

hipError_t launch_residual_f32A(const float2* A, size_t lda, int n, const double2* X, size_t ldx, int nrhs,
                                const double2* B, size_t ldb, double2* R, size_t ldr, double2* partial,
                                hipStream_t s, const KernelHook* hook,
                                const MvShapes* shapes)
{
    return matvec_any<float2, double2, double2, double2>(A, lda, n, X, ldx, nrhs, R, ldr, partial, B, ldb, s, hook,
                                                         shapes);
}


// ---------------------------------------------------------------------------
// Tuning table access (bem_tune and its export / import).
// ---------------------------------------------------------------------------
void force_shape(const MvShape* s) { g_forced = s; }

MvShape current_shape(int types, int ng, int n) { return shape_from(nullptr, types, ng, n); }

std::shared_ptr<const ShapeSnapshot> snapshot_shapes()
{
    auto snap = std::make_shared<ShapeSnapshot>();
    for (int w = 0; w < 2; ++w) snap->have_env[w] = env_shape(w ? 2 : 1, snap->env[w]);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    snap->table = g_tuned;
    return snap;
}

void resolve_shapes(const ShapeSnapshot* snap, int n, MvShapes& out)
{
    for (int t = 0; t < 4; ++t)
        for (int ng = 0; ng <= 4; ++ng) out.s[t][ng] = shape_from(snap, t, ng, n);
}

std::vector<MvShape> candidate_shapes(int types, int ng, int n)
{
    std::vector<MvShape> out;
    const int cap = split_cap(n, ng);
    std::vector<int> splits;
    for (int s = cap; s >= 1; s /= 2) splits.push_back(s);
    if (ng == 0) {
        for (int s : splits) out.push_back(MvShape{0, 0, s, 0});
        return out;
    }
    const MvShape d = mfma_default(n, ng, types & 1);
    out.push_back(d);  // the default first
    const int rts[] = {1, 2, 4}, us[] = {2, 4, 8};
    for (int rt : rts)
        for (int u : us)
            for (int g3 = (ng == 1 ? 0 : 1); g3 <= 1; ++g3)
                for (int s : splits) {
                    const MvShape c{rt, u, s, g3};
                    if (!shape_valid(ng, c)) continue;
                    if (c.rt == d.rt && c.u == d.u && c.g3 == d.g3 && c.splits == d.splits) continue;
                    out.push_back(c);
                }
    return out;
}

void set_tuned_shape(int types, int ng, int n, const MvShape& c)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[ShapeKey{types, ng, size_class(n)}] = c;
}

void clear_tuned_shapes()
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned.clear();
}

std::string export_tuned_shapes()
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    std::ostringstream o;
    o << "# bem product launch shapes: types ng log2n rt u splits g3\n";
    for (const auto& kv : g_tuned)
        o << kv.first.types << ' ' << kv.first.ng << ' ' << kv.first.lg << ' ' << kv.second.rt << ' ' << kv.second.u
          << ' ' << kv.second.splits << ' ' << kv.second.g3 << '\n';
    return o.str();
}

bool import_tuned_shapes(const char* text)
{
    std::map<ShapeKey, MvShape> add;
    std::istringstream in(text ? text : "");
    std::string line;
    while (std::getline(in, line)) {
        if (line.empty() || line[0] == '#') continue;
        std::istringstream l(line);
        ShapeKey k{};
        MvShape c{};
        if (!(l >> k.types >> k.ng >> k.lg >> c.rt >> c.u >> c.splits >> c.g3)) return false;
        std::string rest;
        if (l >> rest) return false;
        if (k.types < 0 || k.types > 3 || k.types == 2 || k.ng < 0 || k.ng > 4 || k.lg < 0 || k.lg > 31) return false;
        if (!shape_valid(k.ng, c)) return false;
        add[k] = c;
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto& kv : add) g_tuned[kv.first] = kv.second;
    return true;
}

}  // namespace bemk
