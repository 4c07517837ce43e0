/*
 * FP64 CPU oracle for the learned-smoother multigrid method of Huang, Li & Xi,
 * "Learning optimal multigrid smoothers via neural networks" (arXiv 2102.12071).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source, header, table or helper with
 * the GPU library.
 *
 * Every routine is the plain definition (or the paper's algorithm in its own
 * order), written for a reader who checks it against the paper by eye:
 * double precision throughout, no blocking, no fusion.  OpenMP is used only
 * to run independent grid rows in parallel.
 *
 * Conventions (shared by every routine):
 *   - Grid: the unit square with an n x n interior, n = 2^k - 1, mesh width
 *     h = 1/(n+1); node (i, j) sits at ((i+1)h, (j+1)h); zero Dirichlet data.
 *   - A grid vector is an array x[j*n + i] (row j is the y index).
 *   - A 9-point stencil field is A[c*n*n + j*n + i], c = 3*(dy+1) + (dx+1):
 *     0 SW, 1 S, 2 SE, 3 W, 4 C, 5 E, 6 NW, 7 N, 8 NE.  Entries that couple
 *     to a node outside the interior are zero.
 *   - A 5x5 smoother stencil field is W[k*n*n + j*n + i], k = 5*(dy+2)+(dx+2).
 *   - Coarse level: n_c = (n-1)/2; coarse node I sits on fine node 2I+1.
 *
 * Parity status of each function is listed beside it ("pinned by" names the
 * independent checks in the test suite).
 */
#ifndef MG_ORACLE_H
#define MG_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- discretisation (paper section 4 stencil; section 6 anisotropic PDE) ---- */

/* Bilinear (Q1) finite-element stencil of -div(K grad u) with a cellwise
 * constant symmetric tensor K = [[k11, k12], [k12, k22]].  Cell (I, J),
 * I, J = 0..n, has its lower-left corner at node (I-1, J-1); the per-cell
 * arrays are [(n+1)*(n+1)] indexed J*(n+1)+I.  The h^-2 factor of the paper is
 * left out: the 2-D stiffness matrix does not depend on h.
 * Pinned by: the paper's section-4 nine-point formula (isotropic cells),
 * an independent Gauss-quadrature element assembly, zero row sums. */
void ora_stencil_q1_cells(int n, const double *k11, const double *k12,
                          const double *k22, double *A);

/* Constant tensor K = R(theta) diag(1, eps) R(theta)^T (strong direction
 * theta), the rotated anisotropic operator of the paper's section 6 with
 * (theta, eps) standing for (theta + pi/2, 1/xi) up to a scale. */
void ora_stencil_q1_rotated(int n, double theta, double eps, double *A);

/* Five-point stencil of -div(a grad u): face coefficients are the mean of the
 * two cells sharing the face; a is per cell, [(n+1)*(n+1)] as above. */
void ora_stencil_cellavg5(int n, const double *a, double *A);

/* ---- operators (section 2: A u = f; section 6: full coarsening) ---- */

/* y = A x, out-of-domain x taken as zero. */
void ora_matvec(int n, const double *A, const double *x, double *y);

/* Full-weighting restriction rc = R r, stencil (1/16)[1 2 1; 2 4 2; 1 2 1]. */
void ora_restrict_fw(int n, const double *r, double *rc);

/* Bilinear prolongation and correction e += P ec (weights 1, 1/2, 1/4). */
void ora_prolong_add(int n, const double *ec, double *e);

/* Galerkin coarse stencil Ac = R A P (n_c = (n-1)/2). */
void ora_galerkin(int n, const double *A, double *Ac);

/* ---- dense coarsest-level solve ---- */

/* Dense matrix [m*m] (row-major) of a stencil field on an n x n grid. */
void ora_stencil_to_dense(int n, const double *A, double *M);
/* In-place Cholesky M = L L^T (lower triangle kept).  Returns 0, or -1 when
 * the matrix is not positive definite. */
int ora_cholesky(int m, double *M);
/* x = (L L^T)^{-1} b. */
void ora_cholesky_solve(int m, const double *L, const double *b, double *x);

/* ---- smoothers (section 2.1 relaxation; section 4 per-point kernels) ---- */

/* One damped-Jacobi sweep e <- e + omega (r - A e) / a_C. */
void ora_smooth_jacobi(int n, const double *A, double omega, const double *r,
                       double *e);
/* One learned-smoother sweep e <- e + H (r - A e) with H applied as a
 * per-point gather stencil, (H x)_p = (1/a_C(p)) sum_k W_p[k] x_{p+k}. */
void ora_smooth_stencil5(int n, const double *A, const double *W,
                         const double *r, double *e);
/* y = H x (the same per-point gather stencil, no residual). */
void ora_apply_smoother5(int n, const double *A, const double *W,
                         const double *x, double *y);

/* ---- multigrid hierarchy, V-cycle (Algorithm 1) and solver ---- */

typedef struct ora_mg ora_mg;

/* Builds levels n, (n-1)/2, ... down to coarsest_n with Galerkin stencils and
 * a Cholesky factor of the coarsest matrix.  Returns NULL on bad sizes or a
 * non-SPD coarsest matrix. */
ora_mg *ora_mg_create(int n, const double *A0, int coarsest_n);
void ora_mg_destroy(ora_mg *mg);
int ora_mg_num_levels(const ora_mg *mg);
int ora_mg_level_n(const ora_mg *mg, int level);
/* Copies the level's stencil field out. */
void ora_mg_get_stencil(const ora_mg *mg, int level, double *A);
/* Installs a 5x5 smoother field W for a level (NULL = damped Jacobi). */
int ora_mg_set_smoother(ora_mg *mg, int level, const double *W);

/* One correction cycle e = V_level(r), with nu1 pre- and nu2 post-sweeps. */
void ora_mg_vcycle(ora_mg *mg, int level, int nu1, int nu2, double omega,
                   const double *r, double *e);

/* Stationary multigrid iteration u_{k+1} = u_k + V(f - A u_k) from u_0 = 0
 * until ||f - A u||_2 / ||f||_2 <= tol or maxit cycles.  history (may be
 * NULL) receives the relative residual after each cycle, [maxit + 1].
 * Returns the number of cycles applied; *converged is set to 0/1. */
int ora_mg_solve(ora_mg *mg, const double *f, double *u, double tol,
                 int maxit, int nu1, int nu2, double omega, double *history,
                 int *converged);

/* ---- the stencil-to-smoother CNN (section 4.2) ---- */

/* Number of parameters of a conv stack with channels ch[0..nlayers]. */
int64_t ora_cnn_num_params(int nlayers, const int *ch);

/* CNN forward on one stencil field: input x0 = A / a_C (9 channels), layers
 * of 3x3 "same" convolutions (zero padding at every layer, PyTorch
 * cross-correlation, weights [Cout][Cin][3][3] followed by bias[Cout]),
 * ReLU after every layer but the last; output W = omega*delta_0 + x_L
 * (delta_0 is 1 in channel 12, the centre of the 5x5 stencil), except on
 * rows whose off-centre entries do not sum to a negative value (Dirichlet
 * nodes of a masked domain and their Galerkin images), where
 * W = omega*delta_0 (damped Jacobi).  W: [25][n][n]. */
void ora_cnn_forward(int n, const double *A, int nlayers, const int *ch,
                     const double *params, double omega, double *W);

/* Mean high-frequency smoothing loss over a batch and its gradient:
 *   L = 1/(B J) sum_b sum_j || v_bj - H_b A_b v_bj ||_2,
 * H_b the per-point smoother produced by the CNN from A_b.
 * ns[b] grid sizes, A[b] stencil fields, V[b] = J vectors [J][n_b*n_b].
 * grad (may be NULL) receives dL/dparams. Returns L. */
/* Vector-Jacobian product of the network: grad += (dW/dparams)^T dW for one
 * problem (A: [9][n][n]; dW: [25][n][n], the gradient of a loss with respect
 * to the network's output W; the omega delta_0 term has no parameters). */
void ora_cnn_vjp(int n, const double *A, int nlayers, const int *ch, const double *params, const double *dW,
                 double *grad);

double ora_hf_loss(int B, const int *ns, const double *const *A,
                   const double *const *V, int J, int nlayers, const int *ch,
                   const double *params, double omega, double *grad);

/* One Adam step (bias-corrected), t = step number starting at 1. */
void ora_adam_step(int64_t np, double *p, double *m, double *v,
                   const double *g, int t, double lr, double beta1,
                   double beta2, double eps);

/* OpenMP threads the routines above use (omp_get_max_threads), and a way to
 * set them (omp_set_num_threads; nthreads >= 1).  Timing aids only: no
 * routine's result depends on the thread count (independent rows). */
int ora_num_threads(void);
void ora_set_threads(int nthreads);

#ifdef __cplusplus
}
#endif
#endif
