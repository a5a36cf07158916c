/*
 * bem_oracle.h -- plain, slow, single-threaded FP64 CPU oracle for the
 * collocation BEM of the Calderon-ordered Burton-Miller transmission problem
 * (Matsumoto, Yoshiki, Isakari, "Automatically well-conditioned collocation
 * boundary element method for transmission problems based on the
 * Burton-Miller formulation", arXiv 2312.12787).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP path.  Only
 * the test-suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.  The product library shares no code, header, table or constant
 * with it and never calls it.
 *
 * Conventions (paper Sec. 2 and Sec. 3.3):
 *   - time factor exp(-i w t), fundamental solution G_k(r) = (i/4) H0^(1)(k r);
 *   - interface m is a polyline of nodes; element e runs from node e to node
 *     e+1 (closed curves wrap); its unit normal is the LEFT normal of the
 *     travel direction and points INTO domain dom_left[m] and OUT of domain
 *     dom_right[m];  the exterior host medium is domain 0;
 *   - eps_d = (k_d / k_0)^2 (paper Sec. 2: k_i = w sqrt(eps_i), eps_1 = 1);
 *   - unknowns x = [u over all elements ; w over all elements], w = (1/eps) du/dn;
 *   - matrices are column-major complex128 with leading dimension 2*N.
 *
 * All complex arrays are interleaved (re, im) doubles, i.e. C99 double complex.
 */
#ifndef BEM_ORACLE_H
#define BEM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Formulation presets.
 *   OR_CALDERON      : eq. (calderon_bieb) with beta=-alpha and, for several
 *                      materials, eq. (3dom_calderon_bie) with gamma_i =
 *                      alpha/eps_i (the recipe at the end of Sec. 6).
 *   OR_CALDERON_BETA1: eq. (calderon_bie1), beta = 1.
 *   OR_CONVENTIONAL  : eq. (naive_bie) / eq. (3dom_conv_bie).
 *   OR_CALDERON_ORIG : eq. (3dom_calderon_bie0): only the host medium uses the
 *                      Burton-Miller equation.                                  */
enum { OR_CALDERON = 0, OR_CALDERON_BETA1 = 1, OR_CONVENTIONAL = 2, OR_CALDERON_ORIG = 3 };

typedef struct or_problem or_problem;

/* Gauss-Legendre rule on [-1,1] by Newton iteration on P_q (Sec. 7 uses it). */
int or_gauss_legendre(int q, double *xi, double *w);

/* Hankel functions of the first kind H0^(1)(z), H1^(1)(z), Im z >= 0, z != 0.
 * out[0..1] = H0 (re, im), out[2..3] = H1 (re, im).                        */
int or_hankel01(double zr, double zi, double *out);

/* Self-terms of a straight element of length h at its own midpoint
 * (out[0..1] = S_ii, out[2..3] = N_ii, finite part).                       */
int or_self_terms(double kr, double ki, double h, double *out);

/* Build a problem.  k: n_dom complex wavenumbers (interleaved); xy: all node
 * coordinates of all interfaces concatenated as (x, y) pairs.  alpha / beta
 * may be NULL (defaults -i/k0 and -alpha, or 1 for the beta=1 / conventional
 * forms); bm_coef may be NULL (defaults alpha/eps_d per domain).          */
or_problem *or_problem_new(int n_dom, const double *k, int n_if, const int *n_nodes,
                           const int *closed, const double *xy, const int *dom_left,
                           const int *dom_right, int quad, int form, const double *alpha,
                           const double *beta, const double *bm_coef);
void or_problem_free(or_problem *p);
int or_n_elements(const or_problem *p);
const char *or_last_error(void);

/* Element table, 9 doubles per element: a(2) b(2) c(2) t(2) h. */
int or_elements(const or_problem *p, double *out);
/* Per element normal (2 doubles). */
int or_normals(const or_problem *p, double *out);

/* Layer-operator entries of domain d between collocation point of element i and
 * element j (global element indices):  out = S, D, Dstar, N  (4 complex).    */
int or_operator_entries(const or_problem *p, int d, int i, int j, double *out);

/* Full system matrix, column-major, 2N x 2N complex. */
int or_assemble(const or_problem *p, double *A);
/* Selected rows: out is nrows x 2N row-major complex (row r at out + r*2N). */
int or_assemble_rows(const or_problem *p, int nrows, const int *rows, double *out);

/* Right-hand sides for plane waves exp(i k0 (cos th, sin th).x):
 * B column-major 2N x nang. */
int or_rhs(const or_problem *p, int nang, const double *angles, double *B);

/* y = A x, A column-major n x n. */
void or_matvec(int n, const double *A, const double *x, double *y);

/* Dense LU with partial pivoting; solves A X = B in place (B n x nrhs col-major).
 * A is overwritten by its factors.  Returns 0, or 1 if a pivot is exactly 0.  */
int or_lu_solve(int n, double *A, int nrhs, double *B);

/* Restarted GMRES(m) with modified Gram-Schmidt and Givens rotations, x0 = 0.
 * Stops when ||b - A x|| <= tol ||b|| (checked on the true residual at each
 * restart and at exit).  iters = number of matrix-vector products with A.
 * Returns 0 when converged, 1 otherwise.                                     */
int or_gmres(int n, const double *A, const double *b, int m, double tol, int max_it,
             double *x, int *iters, double *relres);

/* Far-field pattern of the scattered field in the host medium for solutions X
 * (2N x nrhs col-major): F (ndir x nrhs col-major).                          */
int or_farfield(const or_problem *p, int nrhs, const double *X, int ndir, const double *dirs,
                double *F);

/* Near field (Sec. 7.1) at npts points xy (2 per point) lying in domains
 * dom[npts], for solutions X (2N x nrhs col-major): U (npts x nrhs col-major,
 * complex).  angles[nrhs] (or NULL: scattered field only) adds the incident
 * plane wave at host-medium points.  Returns 1 for a domain out of range.  */
int or_nearfield(const or_problem *p, int nrhs, const double *X, const double *angles, int npts,
                 const double *xy, const int *dom, double *U);

#ifdef __cplusplus
}
#endif
#endif
