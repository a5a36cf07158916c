// launch.h -- host-side entry points of the gfx950 kernels.
#pragma once

#include <memory>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "internal.h"

namespace bemk {

// Optional callback around the main kernel of a launcher (phase 0 before the
// launch, 1 after), used by the library's HIP-event timing.
enum { KIND_ASSEMBLE = 0, KIND_MATVEC = 1, KIND_RESIDUAL = 2, N_KINDS = 3 };
// GMRES stopping-flag read-back: ring of pinned slots and events (host lag + 1)
constexpr int FLAG_RING = 5;
// Graph-captured Arnoldi: at most this many Krylov steps per captured segment
// (the flag ring of that path has GRAPH_MAX_STEPS + 1 slots)
constexpr int GRAPH_MAX_STEPS = 16;
struct KernelHook {
    void (*fn)(void* ctx, int kind, int phase, hipStream_t s);
    void* ctx;
};
inline void hook_call(const KernelHook* h, int kind, int phase, hipStream_t s)
{
    if (h && h->fn) h->fn(h->ctx, kind, phase, s);
}

hipError_t launch_setup(char* g, const GeomLayout& L, int N, int n_dom, int q, hipStream_t s);
// Assembly variants: v = side * 4 + burton_miller * 2 + complex_k; lists[v]
// (device) holds the row-tile ids of variant v, counts[v] (host) their number.
constexpr int ASM_VARIANTS = 8;
// lists[v] / counts[v]: row tiles of variant v (device list / host count);
// pairs[v] / pair_counts[v]: its (row tile, column chunk, part of NEAR_PART
// elements) triples that may hold near element pairs (device list / host count).
// Variants go alternately to s and s1 (they write disjoint rows; s1 may be s).
hipError_t launch_assemble_f64(const char* g, const GeomLayout& L, int N, int n_if, int n_cchunks, int q,
                               const int* const* lists, const int* counts, const int* const* pairs,
                               const int* pair_counts, double2* A, size_t lda, float2* A32, size_t lda32,
                               hipStream_t s, hipStream_t s1);
hipError_t launch_assemble_f32(const char* g, const GeomLayout& L, int N, int n_if, int n_cchunks, int q,
                               const int* const* lists, const int* counts, const int* const* pairs,
                               const int* pair_counts, float2* A, size_t lda, hipStream_t s, hipStream_t s1);

// angles / dirs are HOST arrays: they travel to the kernels by value in
// chunks of ANGLE_CHUNK.
constexpr int ANGLE_CHUNK = 256;
struct AngleChunk {
    double v[ANGLE_CHUNK];
};
hipError_t launch_rhs(const char* g, const GeomLayout& L, int N, const double* angles, int nang, double2* B,
                      size_t ldb, hipStream_t s);

// Y = A X; partial holds matvec_part_elems(n, nrhs) complex values (enough for
// any launch shape), or matvec_part_elems_shaped(shapes, types, n, nrhs) for
// the shapes given (types as in the shape classes below).
size_t matvec_part_elems(int n, int nrhs);
struct MvShapes;
size_t matvec_part_elems_shaped(const MvShapes& sh, int types, int n, int nrhs);

// Launch shape of a product: row tiles per wave, column steps in flight,
// column splits, 3-product form (the vector kernel uses splits only).  Shape
// classes: types = 2 [matrix in FP64] + [accumulation in FP64], ng = 0 (vector
// kernel) or 1-4 groups of 16 right-hand sides, ceil(log2 n).
struct MvShape {
    int rt, u, splits, g3;
};
// The shapes one problem's products run with, by [types][ng], resolved once
// (at assembly) from a source of shapes: the process's tuned table and the
// BEM_MV_CFG / BEM_MV_CFG_WIDE overrides as they are then, or a frozen copy
// of both (the request server's, taken when it is created).  Products never
// read the live table, so a later bem_tune / bem_tune_import or a changed
// environment cannot change the numerics of a problem already assembled.
struct MvShapes {
    MvShape s[4][5];
};
struct ShapeSnapshot;
std::shared_ptr<const ShapeSnapshot> snapshot_shapes();
void resolve_shapes(const ShapeSnapshot* snap /* nullptr: the live table and environment */, int n, MvShapes& out);
void force_shape(const MvShape* s);  // this thread's products use s (nullptr: the resolved shapes again)
MvShape current_shape(int types, int ng, int n);
std::vector<MvShape> candidate_shapes(int types, int ng, int n);
void set_tuned_shape(int types, int ng, int n, const MvShape& c);
void clear_tuned_shapes();
std::string export_tuned_shapes();
bool import_tuned_shapes(const char* text);
hipError_t launch_matvec_f64(const double2* A, size_t lda, int n, const double2* X, size_t ldx, int nrhs,
                             double2* Y, size_t ldy, double2* partial, hipStream_t s,
                             const KernelHook* hook = nullptr, const MvShapes* shapes = nullptr);
// FP32 matrix and products with FP64 vectors: X is rounded to FP32 when packed,
// Y widened when the split partial sums are added.
hipError_t launch_matvec_f32x64(const float2* A, size_t lda, int n, const double2* X, size_t ldx, int nrhs,
                                double2* Y, size_t ldy, float2* partial, hipStream_t s,
                                const KernelHook* hook = nullptr, const MvShapes* shapes = nullptr);
// The same with an FP32 X (a complex64 Krylov basis vector); Y in FP64.
hipError_t launch_matvec_f32v(const float2* A, size_t lda, int n, const float2* X, size_t ldx, int nrhs,
                              double2* Y, size_t ldy, float2* partial, hipStream_t s,
                              const KernelHook* hook = nullptr, const MvShapes* shapes = nullptr);
hipError_t launch_matvec_f32(const float2* A, size_t lda, int n, const float2* X, size_t ldx, int nrhs, float2* Y,
                             size_t ldy, float2* partial, hipStream_t s, const KernelHook* hook = nullptr, const MvShapes* shapes = nullptr);
// The products of the Krylov steps with more than 4 right-hand sides: the
// matrix-core kernel reads them packed at part + xt_offset (XT[c * xw + r],
// zero for nr <= r < xw), written there by the kernel that produced the basis
// vector (start of a cycle, end of the previous step), and its split partial
// sums are added in split order into Y (FP64).
struct ProductPlan {
    MvShape shape;
    int ng, splits, xw;
    size_t xt_offset;  // in complex values of the accumulation type
};
ProductPlan product_plan(const MvShapes* shapes, int types, int n, int nr);
// The normalisation of Krylov step j folded into its product (steps j >= 1
// of a problem whose products read packed right-hand sides): the packed
// inputs hold w of step j - 1 (written by the update kernel), and the split
// reduction divides the product of each right-hand side by |w|, stores
// v_j = w / |w| into the basis, |w| into hnorm and clears the stopping marks
// of step j - 1.
struct StepNorm {
    const double* norm_part;  // [nr][nu] partial sums of |w|^2 of the update blocks
    int nu;                   // update_blocks(n)
    void* V;                  // v_j, column-major (ldv): complex64 if v32, else complex128
    size_t ldv;
    bool v32;
    double* hnorm;
    int* active;
};
int update_blocks(int n);
hipError_t launch_product_packed_f64(const ProductPlan& pl, const double2* A, size_t lda, int n, int nr,
                                     double2* part, double2* Y, size_t ldy, const StepNorm* sn, hipStream_t s,
                                     const KernelHook* hook);
// FP32 matrix and sums (complex64 basis), Y widened to FP64.
hipError_t launch_product_packed_f32(const ProductPlan& pl, const float2* A, size_t lda, int n, int nr,
                                     float2* part, double2* Y, size_t ldy, const StepNorm* sn, hipStream_t s,
                                     const KernelHook* hook);
// R = B - A X (FP64)
hipError_t launch_residual_f64(const double2* A, size_t lda, int n, const double2* X, size_t ldx, int nrhs,
                              const double2* B, size_t ldb, double2* R, size_t ldr, double2* partial, hipStream_t s,
                              const KernelHook* hook = nullptr, const MvShapes* shapes = nullptr);
// R = B - A X with an FP32 matrix, FP64 vectors and FP64 accumulation.
hipError_t launch_residual_f32A(const float2* A, size_t lda, int n, const double2* X, size_t ldx, int nrhs,
                                const double2* B, size_t ldb, double2* R, size_t ldr, double2* partial,
                                hipStream_t s, const KernelHook* hook = nullptr, const MvShapes* shapes = nullptr);

// GMRES building blocks (basis V[(i * nr + r) * ldv + q], FP64).
hipError_t launch_col_norms(const double2* X, size_t ldx, int n, int nr, double* partial, double* out,
                            hipStream_t s);
// Row chunks of the projection kernel and blocks of the update kernel: the
// partial-sum buffers hold arnoldi_blocks(n) entries per right-hand side.
int arnoldi_blocks(int n);
// One Arnoldi step j (0..m) of the batched GMRES cycle (linalg.hip): delayed
// re-orthogonalisation, two passes over the basis; W = A V_j for j < m.
struct ArnoldiArgs {
    double2* V;
    size_t ldv;
    int nr, m, n;
    double2* W;
    size_t ldw;
    double2 *partP, *partQ;        // projection partials [nr][ns][m + 1]
    double2 *Hraw, *H;             // Hessenberg as produced / rotated, [nr][m][m + 1]
    double2 *cs, *sn, *gvec;       // Givens rotations, rotated right-hand side
    double *hnorm, *norm_part;     // |w| of the last step, its partials [nr][nu]
    const double* thr;             // absolute stopping thresholds
    int maxit;
    int *iters, *kdim, *active;    // counters and flags (device)
    int* flags_out;                // copy of the stopping flags in pinned host memory (device address)
    bool v32;                      // basis stored as complex64 at V (same element offsets), else complex128
    // where the next product reads its packed right-hand sides (xw columns;
    // nullptr: the vector product reads V itself)
    void* xt;
    int xw;
};
hipError_t launch_arnoldi(const ArnoldiArgs& a, int j, hipStream_t s);
// The same step j for np (<= MAX_FUSED) problems in one set of launches (all
// with the same restart length and basis precision); each problem's results
// are those of launch_arnoldi on it alone.
constexpr int MAX_FUSED = 8;
hipError_t launch_arnoldi_set(const ArnoldiArgs* a, int np, int j, hipStream_t s);

// Host side (bem_api.cpp): bytes of a matrix buffer of order n and leading
// dimension lda in precision prec (a bem_prec value).
size_t matrix_bytes_ld(int prec, size_t n, size_t lda);
// v_0 = R / |R| per active right-hand side (and its packed copy at xt, xw
// columns, for the first product; xt may be nullptr), g = |R| e_0.
hipError_t launch_start_cycle(const double2* R, size_t ldr, int n, int nr, const double* rnorm, int m,
                              double2* V, size_t ldv, double2* gvec, const int* active, double2* xt, int xw,
                              hipStream_t s);
hipError_t launch_start_cycle(const double2* R, size_t ldr, int n, int nr, const double* rnorm, int m,
                              float2* V, size_t ldv, double2* gvec, const int* active, float2* xt, int xw,
                              hipStream_t s);
hipError_t launch_backsolve(int nr, int m, const double2* H, const double2* gvec, const int* kdim, double2* y,
                            hipStream_t s);
// y: [nr][m + 1] (the back-solve's output)
hipError_t launch_xupdate(const double2* V, size_t ldv, int nr, int n, int m, const double2* y, const int* kdim,
                          double2* X, size_t ldx, hipStream_t s);
hipError_t launch_xupdate(const float2* V, size_t ldv, int nr, int n, int m, const double2* y, const int* kdim,
                          double2* X, size_t ldx, hipStream_t s);
hipError_t launch_axpby_res(const double2* B, size_t ldb, const double2* AX, size_t ldax, int n, int nr,
                            double2* R, size_t ldr, hipStream_t s);
hipError_t launch_add_f64(const double2* D, size_t ldd, int n, int nr, double2* X, size_t ldx, const int* active,
                          hipStream_t s);

// Field at points (nearfield.hip): right-hand sides in groups of NF_RB, their
// angles by value; dom_cplx[d] (host) = domain d has a complex wavenumber.
constexpr int NF_RB = 8;
struct NearAngles {
    double v[NF_RB];
};
hipError_t launch_nearfield(const char* g, const GeomLayout& L, int n_if, int n_dom, int N, int q, const int* dom_cplx,
                            const double2* X, size_t ldx, int nrhs, const double* angles, const double* xy,
                            const int* dom, int npts, double2* U, size_t ldu, hipStream_t s);
hipError_t launch_farfield(const char* g, const GeomLayout& L, int N, int n_if, int n_dom, const double2* X,
                           size_t ldx, int nrhs, const double* dirs, int ndir, double2* F, size_t ldf,
                           hipStream_t s);

}  // namespace bemk
