/*
 * bem.h -- C ABI of the MI355X (gfx950) hot path of the collocation boundary
 * element method for 2-D Helmholtz transmission problems of Matsumoto,
 * Yoshiki and Isakari, "Automatically well-conditioned collocation boundary
 * element method for transmission problems based on the Burton-Miller
 * formulation" (arXiv 2312.12787).
 *
 * The library assembles the dense complex collocation matrix of the
 * Calderon-ordered Burton-Miller system on the GPU and solves it with
 * restarted GMRES whose dense matrix-vector products, Arnoldi projections,
 * norms and Givens updates all run in HIP kernels.
 *
 * Conventions shared by every call (paper Sec. 2, Sec. 3.3, Sec. 6):
 *   - time factor exp(-i w t); fundamental solution G_k(r) = (i/4) H0^(1)(k r);
 *   - domain 0 is the unbounded host medium, k[0] real and > 0; every other
 *     domain d has a wavenumber with Im k[d] >= 0 and eps_d = (k[d]/k[0])^2;
 *   - an interface is a polyline of nodes; element e joins node e to node e+1
 *     (a closed interface also joins its last node to its first); the unit
 *     normal of an element is the LEFT normal of its direction of travel and
 *     points INTO domain dom_left and OUT of domain dom_right; the host
 *     medium must be a dom_right (the normal leaves the host medium, Sec. 2);
 *   - constant elements, collocation at element midpoints, q-point
 *     Gauss-Legendre quadrature off the diagonal, analytic self terms (Sec. 7);
 *   - N_tot = total number of elements; the system order is n = 2 N_tot;
 *     unknowns are [u on every element ; w = (1/eps) du/dn on every element];
 *     for the Calderon forms the standard-type equations fill rows [0, N_tot)
 *     and the Burton-Miller-type ones rows [N_tot, n), both in element order
 *     (closing recipe of Sec. 6);
 *   - every matrix and vector on the device is column-major; complex numbers
 *     are interleaved (re, im) pairs: complex128 for BEM_F64, complex64 for
 *     BEM_F32;
 *   - the library never allocates device memory: the caller passes every
 *     device buffer (sizes from bem_sizes) and owns it (the one exception is
 *     the fixed scratch array of bem_matvec_noalloc, part of the library's
 *     code on each GPU); pointers named *_dev are device pointers, all others
 *     are host pointers;
 *   - all device work of a call is ordered on the caller's stream; calls that
 *     return data to the host (bem_solve) synchronise that stream;
 *   - errors are returned as status codes; bem_last_error() gives a message
 *     for the calling thread.  No call aborts or throws.
 */
#ifndef BEM_H
#define BEM_H

#include <stddef.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bem_problem bem_problem;

typedef struct {
    double re, im;
} bem_z;

typedef enum {
    BEM_OK = 0,
    BEM_E_ARG = 1,       /* an argument is out of range or inconsistent            */
    BEM_E_GEOMETRY = 2,  /* invalid boundary description                          */
    BEM_E_STATE = 3,     /* call order violated (e.g. matvec before assemble)      */
    BEM_E_DEVICE = 4,    /* a HIP call failed; message in bem_last_error()         */
    BEM_E_NOMEM = 5,     /* a caller buffer is smaller than bem_sizes asked for    */
    BEM_E_NOCONV = 6,    /* GMRES stopped at max_iter; X holds the last iterate   */
    BEM_E_NONFINITE = 7  /* NaN or Inf met in a residual                           */
} bem_status;

/* Matrix precision.
 *   BEM_F64    complex128 matrix; FP64 products.
 *   BEM_F32    complex64 matrix (FP32 assembly with FP64 distances, phases,
 *              small-argument series and self terms); FP32 products, FP64
 *              Arnoldi, refinement residuals with the FP32 matrix (FP64
 *              accumulation): converges to the solution of the FP32 matrix.
 *   BEM_MIXED  the complex128 matrix followed, at byte offset
 *              256-aligned(16 n lda), by its complex64 rounding (same lda),
 *              both written by one assembly pass; FP32 products on the copy,
 *              refinement residuals with the FP64 matrix: converges to the
 *              solution of the FP64 matrix (iterative refinement with the
 *              residual in FP64), for problems whose condition number would
 *              amplify FP32 matrix rounding beyond the target.            */
typedef enum { BEM_F64 = 0, BEM_F32 = 1, BEM_MIXED = 2 } bem_prec;

/* Formulation presets.
 *   BEM_CALDERON       eq. (calderon_bieb) with beta = -alpha for one inclusion,
 *                      eq. (3dom_calderon_bie) with gamma_d = alpha/eps_d for
 *                      several (the recipe closing Sec. 6).  Default.
 *   BEM_CALDERON_BETA1 eq. (calderon_bie1) (beta = 1).
 *   BEM_CONVENTIONAL   eq. (naive_bie) / eq. (3dom_conv_bie): equations listed
 *                      domain by domain, host medium first, unscaled.
 *   BEM_CALDERON_ORIG  eq. (3dom_calderon_bie0): only the host medium uses the
 *                      Burton-Miller equation.                                   */
typedef enum {
    BEM_CALDERON = 0,
    BEM_CALDERON_BETA1 = 1,
    BEM_CONVENTIONAL = 2,
    BEM_CALDERON_ORIG = 3
} bem_form;

/* Problem statement (Sec. 2): domains with their wavenumbers, interfaces
 * between them, and the coupling constants of the Burton-Miller equations.
 * All pointers are host pointers, read during bem_create only.              */
typedef struct {
    int n_dom;              /* number of domains, >= 2                                  */
    const bem_z *k;         /* [n_dom] wavenumbers; k[0] real > 0; Im k[d] >= 0         */
    int n_if;               /* number of interfaces, >= 1                               */
    const int *n_nodes;     /* [n_if] nodes of each interface                           */
    const int *closed;      /* [n_if] 1: closed curve (>= 3 nodes), 0: open (>= 2 nodes) */
    const double *xy;       /* [2 * sum(n_nodes)] node coordinates (x, y), interface by interface */
    const int *dom_left;    /* [n_if] domain the normal points into (never 0)           */
    const int *dom_right;   /* [n_if] domain the normal leaves                          */
    int quad;               /* Gauss-Legendre points per element, 1..16 (8 or 10 usual) */
    int form;               /* bem_form                                                 */
    const bem_z *alpha;     /* NULL: -i / k[0] (Sec. 3.3)                               */
    const bem_z *beta;      /* NULL: -alpha for BEM_CALDERON / BEM_CALDERON_ORIG, else 1 */
    const bem_z *bm_coef;   /* [n_dom] or NULL: Burton-Miller coefficient alpha/eps_d   */
} bem_desc;

/* Validate a problem statement and build its host-side plan (element and row
 * bookkeeping).  No device work.  On success *out owns the plan; free it with
 * bem_destroy.  BEM_E_GEOMETRY: too few nodes, a zero-length element, an
 * unknown or repeated domain id, the host medium on the normal's side, or
 * |1 + eps_left/eps_right| < 1e-12 (accumulation point at 0, end of Sec. 5).
 * BEM_E_ARG: k[0] not real-positive, Im k < 0, a lossy wavenumber with
 * arg k > 10 degrees (Im k > tan(10 deg) Re k: the device's large-argument
 * Hankel form continues real-axis amplitude fits to complex arguments, with a
 * relative error of 1e-14 at arg k = 3.2 deg and 1.7e-12 at 10 deg), quad out
 * of range, or max |k| times the diameter of the nodes' bounding box >= 2^29
 * (the device reduces phases k r by pi/2 exactly only below 2^30).           */
bem_status bem_create(const bem_desc *desc, bem_problem **out);
void bem_destroy(bem_problem *p);

/* Number of elements N_tot and system order n = 2 N_tot. */
int bem_n_elements(const bem_problem *p);
int bem_order(const bem_problem *p);

/* Byte sizes of the caller-owned device buffers:
 *   geom_bytes   geometry / quadrature / constant tables (bem_geometry),
 *   matrix_bytes the n x n matrix at lda = n in precision prec,
 *   work_bytes   workspace of bem_matvec, bem_solve and bem_farfield for up to
 *                nrhs right-hand sides, GMRES restart length `restart` and up
 *                to 4096 far-field directions.  Any pointer may be NULL.     */
bem_status bem_sizes(const bem_problem *p, int prec, int nrhs, int restart, size_t *geom_bytes,
                     size_t *matrix_bytes, size_t *work_bytes);

/* Step (boundary -> element tables), Sec. 4 and Sec. 7: upload the nodes and
 * the plan into geom_dev and compute on the device the element table
 * (end nodes, midpoint, tangent, left normal, length), the Gauss-Legendre
 * rule, the Gauss points of every element, the per-domain constants (eps,
 * Burton-Miller coefficients, Hankel-function tables) and the analytic
 * self terms.  geom_dev must stay alive (and unmodified) until the problem is
 * destroyed or bem_geometry is called again.                                 */
bem_status bem_geometry(bem_problem *p, void *geom_dev, size_t geom_bytes, hipStream_t stream);

/* Recompute every derived device table of bem_geometry (element table, Gauss
 * rule and points, per-domain constants, self terms) from the inputs already
 * uploaded into geom_dev, with no host-to-device copy and no synchronisation.
 * Invalidates the recorded matrix (bem_assemble must run again).            */
bem_status bem_geometry_update(bem_problem *p, hipStream_t stream);

/* Assemble the n x n system matrix (eqs. (stmp)-(ddtmp), (fundamental_sol),
 * the block systems of Secs. 3-6) into A_dev with leading dimension lda >= n,
 * in precision prec (BEM_F64: complex128; BEM_F32: complex64 entries, with
 * self terms computed in FP64 and rounded; BEM_MIXED: complex128 and its
 * complex64 rounding, layout under bem_prec).  Requires bem_geometry.  The
 * problem records A_dev, lda and prec for bem_matvec / bem_solve.  An lda
 * whose columns start on 128-byte lines (a multiple of 8 entries for
 * complex128, 16 for complex64) lets the products read each column segment
 * without a partial line; a buffer with lda > n needs lda / n times the
 * bem_sizes matrix bytes (for BEM_MIXED: the FP64 part, rounded up to 256
 * bytes, then lda * n complex64).                                           */
bem_status bem_assemble(bem_problem *p, int prec, void *A_dev, size_t lda, hipStream_t stream);

/* Right-hand sides of the plane waves exp(i k0 (cos th, sin th) . x), one per
 * angle (host array angles[nang]): u_in + alpha q_in on the rows of the host
 * medium's Burton-Miller equation, 0 elsewhere (eq. (calderon_bieb)).  B_dev
 * is complex128, n x nang, leading dimension ldb >= n.                      */
bem_status bem_rhs(const bem_problem *p, int nang, const double *angles, void *B_dev, size_t ldb,
                   hipStream_t stream);

/* Y = A X for nrhs columns (the dense products of GMRES, Sec. 3.2).  X and Y
 * have the precision of the assembled matrix (complex128 for BEM_F64 and
 * BEM_MIXED, whose FP64 matrix is used; complex64 for BEM_F32), leading
 * dimensions ldx, ldy >= n.  work_dev holds
 * split-K partial sums (bem_sizes with this nrhs).                          */
bem_status bem_matvec(const bem_problem *p, int nrhs, const void *X_dev, size_t ldx, void *Y_dev,
                      size_t ldy, void *work_dev, size_t work_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): bem_matvec
 * without a workspace argument.  The split-K partial sums and the packed
 * right-hand sides live in a device array of BEM_NOALLOC_SCRATCH_BYTES that
 * the library holds on every GPU it runs on until the process ends (its
 * address is looked up once per device, on the first call with that device
 * current; the current device must be the stream's).  Same kernels, launch
 * shapes and summation order as bem_matvec, hence the same Y.  The call
 * allocates nothing and never records timing events (bem_profile_enable does
 * not apply).  BEM_E_ARG when the product's partial sums would exceed the
 * array (FP64: about splits x nrhs x n x 16 bytes, e.g. n = 8192 with 16
 * right-hand sides in the built-in shape takes 18.9 MB); every other error as
 * bem_matvec.  All calls on one GPU share the array: calls that overlap in
 * time on that GPU (other streams, other threads) race and give wrong
 * results; calls ordered on one stream are safe.  Nothing in the array needs
 * clearing between calls (every call writes what it reads).                 */
#define BEM_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
bem_status bem_matvec_noalloc(const bem_problem *p, int nrhs, const void *X_dev, size_t ldx, void *Y_dev,
                              size_t ldy, hipStream_t stream);

/* Largest GMRES restart length: a cycle's Hessenberg column, rotations and
 * projection sums of one right-hand side live in one workgroup's LDS
 * (5 (m + 1) complex128 values plus 4.4 KB, at most 160 KB on gfx950).    */
#define BEM_MAX_RESTART 1990

typedef struct {
    int restart;        /* GMRES restart length m, 1..BEM_MAX_RESTART                    */
    int max_iter;       /* cap on matrix-vector products per right-hand side            */
    double tol;         /* stop when ||b - A x|| <= tol ||b|| (true residual, FP64)      */
    double inner_tol;   /* BEM_F32 / BEM_MIXED only: relative tolerance of each inner solve;
                           0 selects 1e-5                                               */
    int max_refine;     /* BEM_F32 / BEM_MIXED only: cap on FP64 refinement steps; 0 -> 20 */
    int graph_steps;    /* 0: every Krylov step is launched kernel by kernel.  1..16: the
                           steps run as captured HIP graphs of graph_steps steps each
                           (product + orthogonalisation kernels), captured on first use
                           and replayed in later cycles and calls; the host reads the
                           device-side stopping flags one segment late, so up to about
                           2 graph_steps products past a column's stop are spent.  Same
                           kernels and order as 0, hence the same X.  The graphs keep the
                           matrix, work buffer, nrhs, restart, max_iter and product launch
                           shapes they were captured with; a call that changes any of
                           them (a new assembly that resolved other shapes, or a
                           bem_tune of this problem, included) captures again.
                           Ignored while bem_profile_enable is on.                   */
} bem_solve_opts;

typedef struct {
    int iters;          /* Krylov steps (one product each) summed over restart cycles    */
    int restarts;       /* restart cycles (FP64) or refinement steps (BEM_F32, BEM_MIXED) */
    int converged;      /* 1 if the true relative residual reached tol                   */
    double rel_residual;/* final true relative residual ||b - A x|| / ||b||              */
} bem_solve_info;

/* Solve A X = B for nrhs right-hand sides (complex128, n x nrhs, ldb >= n) by
 * GMRES(restart) started from X = 0 (Sec. 3.2: the Krylov space of A itself,
 * no preconditioner applied).  The right-hand sides share every matrix pass
 * (block products); their Krylov spaces are independent.  The Arnoldi
 * process orthogonalises each new vector once and re-orthogonalises it one
 * step later in the same pass (two passes over the basis per step; each
 * cycle spends one extra product on the step at which it stops).  With a
 * BEM_F32 or BEM_MIXED matrix the inner GMRES runs FP32 products and FP64
 * Arnoldi, and an outer FP64 iterative refinement recomputes r = b - A x
 * with FP64 accumulation (FP32 matrix for BEM_F32, FP64 matrix for
 * BEM_MIXED) until tol.  X_dev is complex128 (ldx >= n) and is overwritten.  info is a host
 * array [nrhs].  Returns BEM_E_NOCONV if any column missed tol.            */
bem_status bem_solve(bem_problem *p, int nrhs, const void *B_dev, size_t ldb, const bem_solve_opts *opts,
                     void *X_dev, size_t ldx, void *work_dev, size_t work_bytes, bem_solve_info *info,
                     hipStream_t stream);

/* bem_solve for np (1..8) distinct problems at once, on one stream, with the
 * same options: their restart cycles run in step, each Krylov step launching
 * every problem's product and then one fused set of orthogonalisation
 * kernels (projections, Arnoldi step, update, normalisation) for all of them;
 * a problem whose columns have all stopped drops out of the steps, and at a
 * cycle end each problem restarts or finishes on its own (mixed precision:
 * the outer refinement steps run in step as well).  Every argument is an
 * array over the problems (host arrays of np entries; ps[k], B_dev[k],
 * X_dev[k], work_dev[k], info[k] as the same arguments of bem_solve).  The
 * problems must all be BEM_F64 or all FP32-product (BEM_F32 / BEM_MIXED).
 * Each problem's X and info are bit-identical to those of bem_solve on it
 * alone (the fused kernels run each problem's arithmetic in the same order);
 * graph_steps is ignored for np > 1.  Returns the first error met, or
 * BEM_E_NONFINITE / BEM_E_NOCONV if any column of any problem met it.      */
bem_status bem_solve_batch(int np, bem_problem *const *ps, const int *nrhs, const void *const *B_dev,
                           const size_t *ldb, const bem_solve_opts *opts, void *const *X_dev, const size_t *ldx,
                           void *const *work_dev, const size_t *work_bytes, bem_solve_info *const *info,
                           hipStream_t stream);

/* Far-field pattern of the scattered field in the host medium for nrhs
 * solutions (complex128 X_dev, ldx >= n): u_sc ~ e^{i k0 |x|} / sqrt|x| F,
 *   F(th) = e^{i pi/4} / sqrt(8 pi k0) sum_j sigma_j [w_j + i k0 (xh.n_j) u_j]
 *           h_j e^{-i k0 xh.c_j} sinc(k0 h_j xh.t_j / 2)
 * over the elements of the host medium's boundary (sigma_j = +1 when the
 * normal leaves the host medium).  dirs: host array of ndir <= 4096 angles.
 * F_dev complex128, ndir x nrhs, ldf >= ndir.                               */
bem_status bem_farfield(const bem_problem *p, int nrhs, const void *X_dev, size_t ldx, int ndir,
                        const double *dirs, void *F_dev, size_t ldf, void *work_dev, size_t work_bytes,
                        hipStream_t stream);

/* Field at points off the boundary (Sec. 7.1 evaluates the total field at
 * field points): for a point x of domain d, Green's representation formula
 * of that domain with the solution's boundary data,
 *   u(x) = [d = 0] u_in(x) + sum_m sigma_dm sum_j (eps_d S_j(x) w_j - D_j(x) u_j),
 * S_j, D_j the single- and double-layer integrals of G_d over element j and
 * sigma_dm = +1 where interface m's normal leaves d.  Points at least two
 * element lengths from an element use its Gauss rule; closer ones integrate
 * the Laplace parts of the kernels exactly and the smooth remainder by Gauss.
 * X_dev: nrhs solutions (complex128, ldx >= n).  angles: host [nrhs], the
 * incident angles (adds u_in at host-medium points), or NULL for the
 * scattered field only.  xy_dev: device [2 npts] coordinates; dom_dev: device
 * [npts] domain of each point, chosen by the caller (points with an id outside
 * [0, n_dom) are skipped and their U entries left untouched).  U_dev:
 * complex128 npts x nrhs, point fastest, ldu >= npts.  Requires bem_geometry. */
bem_status bem_nearfield(const bem_problem *p, int nrhs, const void *X_dev, size_t ldx, const double *angles,
                         int npts, const double *xy_dev, const int *dom_dev, void *U_dev, size_t ldu,
                         hipStream_t stream);

/* Kernel timing for measurement.  While enabled, the library records HIP
 * events on the caller's stream immediately before and after the main kernel
 * of every assembly (the fused block-assembly kernel), every dense product
 * Y = A X (the split-K product kernel, not its small reduction pass; including
 * the products inside bem_solve) and every residual product R = B - A X of
 * bem_solve (FP64 accumulation; with an FP32 matrix these are the outer
 * refinement residuals).  bem_profile_read waits for the recorded events,
 * returns the launch counts and summed durations, and with reset != 0 starts
 * a new tally.  Host event objects are created by the library as needed and
 * released by bem_destroy; no device memory is used.                        */
typedef struct {
    int assemble_launches;
    double assemble_ms;
    int matvec_launches;
    double matvec_ms;
    int residual_launches;
    double residual_ms;
} bem_profile;
bem_status bem_profile_enable(bem_problem *p, int on);
bem_status bem_profile_read(bem_problem *p, bem_profile *out, int reset);

/* Launch-shape autotuning of the products inside bem_solve (Sec. 3.2: every
 * Krylov step costs one product with the dense matrix).  bem_tune times each
 * candidate launch shape of that product -- rows per wave, columns in flight,
 * column splits, complex-product form -- with the problem's assembled matrix
 * and nrhs right-hand sides (the FP64 matrix for BEM_F64; the FP32 matrix,
 * or the FP32 copy of BEM_MIXED, with FP64 vectors otherwise), `reps` timed
 * products each after one untimed (the four fastest twice more, each keeping
 * its best time), and installs the fastest for its shape
 * class: (matrix and accumulation precision, right-hand-side groups of 16 up
 * to 64 or the vector kernel's up to 4, ceil(log2 n)) in the process's table.
 * A problem resolves the shapes of all its products when bem_assemble runs
 * (from that table and the BEM_MV_CFG / BEM_MV_CFG_WIDE overrides as they are
 * then) and keeps them until its next bem_assemble: the tuned problem itself
 * switches to the new shape at once, every other problem at its next
 * assembly, so a table change (bem_tune, bem_tune_import, bem_tune_reset)
 * never changes the rounding of the products of a problem already assembled.
 * A request server resolves every request from a copy of the table taken when
 * the server was created (bem_serve.h).  X_dev
 * (complex128, n x nrhs, ldx >= n) is read, Y_dev (same shape, ldy) is
 * overwritten with A X, work_dev as for bem_matvec.  Candidates never need
 * more work memory than bem_sizes reports, before or after tuning.  The call
 * synchronises the stream.  BEM_E_STATE: no matrix; BEM_E_ARG: bad sizes or
 * reps outside [1, 100]; BEM_E_NOMEM: work smaller than bem_sizes asks.      */
typedef struct {
    int rt, u, splits, g3;       /* chosen shape (vector kernel: rt = u = g3 = 0)       */
    int candidates;              /* shapes timed                                        */
    double best_ms, default_ms;  /* average product time: chosen shape, built-in shape  */
} bem_tune_info;
bem_status bem_tune(const bem_problem *p, int nrhs, const void *X_dev, size_t ldx, void *Y_dev, size_t ldy,
                    void *work_dev, size_t work_bytes, int reps, bem_tune_info *info, hipStream_t stream);

/* The tuned shape table as text (one class per line: types ng log2n rt u
 * splits g3; a '#' line first).  Writes at most len bytes including the
 * terminating NUL into buf (may be NULL when len = 0) and returns the length
 * of the whole text (without NUL), so a first call with len = 0 sizes it.   */
size_t bem_tune_export(char *buf, size_t len);
/* Add the classes of a text in bem_tune_export's format to the table (lines
 * starting with '#' are skipped).  BEM_E_ARG and no change on a malformed
 * line or an invalid shape.                                                 */
bem_status bem_tune_import(const char *text);
/* Forget every tuned shape (built-in shapes again). */
void bem_tune_reset(void);

/* Message of the last non-OK status returned on this thread ("" if none). */
const char *bem_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BEM_H */
