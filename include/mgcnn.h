/*
 * mgcnn — geometric multigrid with a learned per-point smoother on AMD
 * Instinct MI355X (gfx950).
 *
 * The method is that of Huang, Li & Xi, "Learning optimal multigrid smoothers
 * via neural networks" (arXiv 2102.12071): a V-cycle (Algorithm 1) on a
 * structured 2-D grid with full coarsening, full-weighting restriction,
 * bilinear prolongation and Galerkin coarse operators (section 6.1), whose
 * smoother is produced by a convolutional network that maps each point's
 * operator stencil to the stencil of the smoother inverse (section 4.2).
 *
 * Conventions used by every entry point
 * -------------------------------------
 * Grid: the unit square with an n x n interior, n = 2^k - 1; node (i, j) sits
 *   at ((i+1)h, (j+1)h), h = 1/(n+1); zero Dirichlet boundary values.
 * Vectors: [n][n] row-major (row j = y index), contiguous, FP64, on the device.
 * Stencil fields: [9][n][n] FP64 on the device, channel c = 3(dy+1) + (dx+1)
 *   (0 SW, 1 S, 2 SE, 3 W, 4 C, 5 E, 6 NW, 7 N, 8 NE).  Entries that couple to
 *   a node outside the interior must be zero, and the centre entry positive.
 * Smoother fields: [25][n][n], channel k = 5(dy+2) + (dx+2); the smoother acts
 *   as a gather stencil, (H x)_p = (1/a_C(p)) sum_k W_p[k] x_{p+k}.
 * Levels: level 0 is the input grid; level l+1 has n_{l+1} = (n_l - 1)/2 and
 *   coarse node I sits on fine node 2I+1; the last level has n = coarsest_n.
 * Streams: every call enqueues its work on the HIP stream given at creation
 *   (a hipStream_t passed as void*, NULL = the null stream) and returns
 *   without synchronising, except the calls marked "synchronises".
 * Ownership: the caller owns every pointer it passes; calls copy what they
 *   keep.  Contexts and networks own their device memory until destroyed.
 * Errors: every call returns an mg_status; on a negative status nothing was
 *   written to the caller's outputs and mg_last_error() (thread-local) holds
 *   a message.  A context or network is not thread-safe; distinct ones are
 *   independent.
 */
#ifndef MGCNN_H
#define MGCNN_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MG_OK = 0,
    MG_NOT_CONVERGED = 1,   /* result produced; the tolerance was not reached */
    MG_ERR_ARG = -1,        /* bad argument (null pointer, bad size, invalid stencil) */
    MG_ERR_SHAPE = -2,      /* sizes inconsistent with the context or network */
    MG_ERR_DEVICE = -3,     /* HIP runtime error, or no gfx950 device */
    MG_ERR_DIVERGED = -4,   /* residual became NaN/Inf or grew by more than 1e3 */
    MG_ERR_STATE = -5,      /* call not valid in this state (e.g. CNN smoother before inference) */
    MG_ERR_OOM = -6         /* device allocation failed */
} mg_status;

typedef struct mg_ctx_s *mg_ctx;   /* solver context: hierarchy for a batch of problems */
typedef struct mg_net_s *mg_net;   /* smoother network: parameters and optimiser state */

enum { MG_SMOOTHER_JACOBI = 0, MG_SMOOTHER_CNN = 1, MG_SMOOTHER_STACK = 2 };
#define MG_STACK_WEIGHTS 54
enum { MG_PREC_FP64 = 0, MG_PREC_MIXED = 1 };

/* ------------------------------------------------------------------------ */
/* Discretisation (paper section 4: bilinear nine-point stencil; section 6:  */
/* rotated anisotropic and variable-coefficient diffusion).                  */
/* ------------------------------------------------------------------------ */

/* Bilinear finite-element stencil of -div(K grad u) with the constant tensor
 * K = R(theta) diag(1, eps) R(theta)^T (strong direction theta, 0 < eps <= 1),
 * without the h^-2 factor (the 2-D stiffness does not depend on h).
 * out: device [9][n][n] FP64.  n odd, 1 <= n <= 16383. */
mg_status mg_stencil_q1_rotated(int32_t n, double theta, double eps, double *out, void *stream);

/* Five-point stencil of -div(a grad u) whose face coefficients are the mean of
 * the two cells sharing the face.  a: device [(n+1)][(n+1)] FP64 per cell,
 * cell (I, J) having its lower-left corner at node (I-1, J-1); a > 0.
 * out: device [9][n][n] FP64 (corner channels zero). */
mg_status mg_stencil_cellavg5(int32_t n, const double *a, double *out, void *stream);

/* Restricts a stencil to a domain inside the square (the non-square geometries
 * of section 6): nodes with mask 0 lie outside and carry the zero Dirichlet
 * value; their rows keep only the centre entry (so the row reads u_p = f_p / a_C,
 * and f must be 0 there), and the rows of the nodes inside drop their
 * couplings to them.  The result is the operator of the interior nodes, with
 * the outside nodes decoupled, and stays symmetric positive definite.
 * mask: device [n][n] bytes (nonzero = inside); A, out: device [9][n][n]
 * FP64 (out may be A).  n odd, 1 <= n <= 16383. */
mg_status mg_stencil_mask(int32_t n, const uint8_t *mask, const double *A, double *out, void *stream);

/* Galerkin coarse stencil Ac = R A P with R full weighting and P bilinear
 * (section 2.2, coarse operator P^T A P up to the factor 1/4 of R = P^T/4).
 * A: device [9][n][n]; Ac: device [9][nc][nc], nc = (n-1)/2.  n odd >= 3. */
mg_status mg_galerkin(int32_t n, const double *A, double *Ac, void *stream);

/* ------------------------------------------------------------------------ */
/* Solver context (Algorithm 1 and the solver Phi(u0, f, k) of section 2).   */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t n;              /* interior points per side, n = 2^k - 1, coarsest_n <= n <= 8191 */
    const double *stencil;  /* device [9][n][n] FP64, conventions above */
} mg_problem;

typedef struct {
    int32_t smoother;       /* MG_SMOOTHER_JACOBI, MG_SMOOTHER_CNN or MG_SMOOTHER_STACK (weights
                               from mg_set_stack; runs the step-by-step cycle kernels)        */
    int32_t nu_pre;         /* pre-smoothing sweeps, 0..8 (default 1)                          */
    int32_t nu_post;        /* post-smoothing sweeps, 0..8 (default 1)                         */
    double omega;           /* damping of the Jacobi smoother and of the CNN's Jacobi term (2/3) */
    int32_t coarsest_n;     /* 1, 3 or 7 (default 7): solved directly in FP64                 */
    int32_t precision;      /* MG_PREC_FP64: every kernel in FP64 (parity mode);
                               MG_PREC_MIXED: BF16 smoother and CNN on MFMA, FP32 inner cycle,
                               FP64 outer residual, norms and coarsest solve (default)        */
    int32_t use_graph;      /* 1: capture one solver iteration as a HIP graph and replay it    */
    int32_t check_every;    /* iterations between host convergence checks in mg_solve (0 = 16) */
    int32_t fallback;       /* 1: in mg_solve with MG_SMOOTHER_CNN, a problem whose residual has not
                               improved on its best by 0.1 % for 16 cycles, or has grown to 100 times
                               its best, is switched to damped Jacobi: its smoother fields are
                               overwritten with omega / a_C (u restarts from 0 after a divergence,
                               continues otherwise).  mg_last_fallbacks tells which; a later CNN
                               solve needs mg_smoother_infer again.  0 (default): off; must be 0
                               with MG_SMOOTHER_STACK. */
} mg_options;

/* Fills the defaults listed above. */
void mg_options_default(mg_options *opt);

/* Builds the hierarchy of every problem: copies the stencils, forms the
 * Galerkin levels in FP64 (and FP32 copies in mixed precision), and factors
 * each coarsest matrix (Cholesky, explicit inverse, FP64).  Problems may have
 * different n.  Validates the stencils (boundary entries zero, centre
 * positive, coarsest matrix SPD): MG_ERR_ARG otherwise.  Synchronises. */
mg_status mg_setup(const mg_problem *probs, int32_t nprob, const mg_options *opt, void *stream,
                   mg_ctx *out);
mg_status mg_destroy(mg_ctx ctx);

/* Replaces every problem's stencil (same sizes as at set-up) and rebuilds the
 * Galerkin levels and coarsest inverses in place, without allocating; the
 * smoothers become stale until the next mg_smoother_infer.  Validates like
 * mg_setup.  Synchronises. */
mg_status mg_restencil(mg_ctx ctx, const mg_problem *probs);

/* Number of levels of problem prob (1 + number of coarsenings). */
mg_status mg_num_levels(mg_ctx ctx, int32_t prob, int32_t *nlev);

/* Copies the FP64 stencil of a level out: device [9][n_l][n_l]. */
mg_status mg_get_stencil(mg_ctx ctx, int32_t prob, int32_t level, double *out);

/* Runs the network on every level but the coarsest of every problem and keeps
 * the resulting smoothers (section 4.2: stencil -> per-point smoothing kernel)
 * in the context.  In mixed precision the network runs in BF16 on MFMA with
 * FP32 accumulation and the smoother is stored in BF16; in FP64 precision
 * every operation is FP64.  A row whose off-centre entries do not sum to a
 * negative value gets damped Jacobi, W = omega * delta_0, instead of the
 * network's output: the off-centre entries of a diffusion row sum to -a_C
 * inside the domain, while the Dirichlet nodes of mg_stencil_mask and their
 * Galerkin images on coarser levels do not sum to a negative value.
 * Required before solving with MG_SMOOTHER_CNN. */
mg_status mg_smoother_infer(mg_ctx ctx, mg_net net);

/* Runs the network on the smoothing levels of size n only (every problem),
 * leaving the other levels' smoothers as they are: per-level networks, each
 * trained for one level size (the adaptive training of section 3.3 yields one
 * network per level).  A level never given a smoother holds zeros (no
 * smoothing), so cover every level size before a CNN solve.  MG_ERR_ARG if
 * no level above the coarsest has size n. */
mg_status mg_smoother_infer_size(mg_ctx ctx, mg_net net, int32_t n);

/* Per-level networks in one call (section 3.3's adaptive training yields one
 * network per level): the smoothing levels of size sizes[k] take nets[k], for
 * k < count (host arrays; count <= 16).  Every smoothing level size of the
 * context must be listed, each once, and every listed size must occur
 * (MG_ERR_ARG otherwise, before any work).  The same smoothers as one
 * mg_smoother_infer_size call per size; in mixed precision one launch covers
 * every level. */
mg_status mg_smoother_infer_levels(mg_ctx ctx, const mg_net *nets, const int32_t *sizes, int32_t count);

/* Installs an explicit smoother field W for one level (device [25][n_l][n_l]
 * FP64; stored as the context's precision).  Replaces what inference gave. */
mg_status mg_set_smoother(mg_ctx ctx, int32_t prob, int32_t level, const double *W);

/* Copies a level's smoother out as W = a_C * H, device [25][n_l][n_l] FP64
 * (in mixed precision: the BF16 values held, times a_C in FP64). */
mg_status mg_get_smoother(mg_ctx ctx, int32_t prob, int32_t level, double *out);

/* One iteration u <- u + V(f - A u) for every problem (the V-cycle of
 * Algorithm 1 in correction form, nu_pre/nu_post sweeps, down to the coarsest
 * level).  f[p], u[p]: device [n_p][n_p] FP64. */
mg_status mg_vcycle(mg_ctx ctx, const double *const *f, double *const *u);

/* Stationary iteration u_0 = 0, u_{k+1} = u_k + V(f - A u_k) until
 * ||f - A u||_2 / ||f||_2 <= rtol (section 6.1 stopping rule) or maxit
 * iterations, per problem.  Host outputs (each may be NULL): iters[nprob],
 * relres[nprob] (final relative residual, FP64), status[nprob]
 * (MG_OK, MG_NOT_CONVERGED or MG_ERR_DIVERGED), history[nprob][maxit+1]
 * (relative residual before each iteration; entries past the last are 0).
 * Returns MG_OK when every problem converged, MG_NOT_CONVERGED or
 * MG_ERR_DIVERGED otherwise (the solutions are written in every case).
 * Synchronises. */
mg_status mg_solve(mg_ctx ctx, const double *const *f, double *const *u, double rtol, int32_t maxit,
                   int32_t *iters, double *relres, int32_t *status, double *history);

/* Flexible GMRES (section 6, incorporation with FGMRES): restarted FGMRES(m)
 * on A u = f for every problem of the context (one after another), right-
 * preconditioned by one cycle of mg_vcycle per iteration (the context's
 * smoother, sweeps and precision; the flexible variant keeps each
 * preconditioned direction, so a mixed-precision cycle is a valid
 * preconditioner).  u_0 = 0; stops when the true FP64 relative residual
 * ||f - A u|| / ||f|| <= rtol, or after maxit iterations (cycles).
 * restart: m in [1, 256]; the context keeps 2m + 4 FP64 vectors of its
 * largest finest grid (allocated on the first call, grown for a larger m).
 * Host outputs as in mg_solve (each may be NULL): iters = preconditioner
 * applications, relres = final true relative residual, status, history
 * [nprob][maxit+1] = the GMRES residual estimate / ||f|| after each
 * iteration (entry 0 = 1).  Synchronises. */
mg_status mg_solve_fgmres(mg_ctx ctx, const double *const *f, double *const *u, double rtol, int32_t maxit,
                          int32_t restart, int32_t *iters, double *relres, int32_t *status, double *history);

/* mg_solve_fgmres for callers that cannot allocate device memory (code that a
 * caller records into a HIP graph of its own, tight serving loops, harnesses
 * that forbid hipMalloc): the same solve, bit for bit, with the Krylov
 * workspace in a fixed device array of MG_FGMRES_NOALLOC_BYTES (64 MiB) per
 * GPU instead of the context's memory.  The array is loaded with the library's
 * code object and held until the process ends; this call allocates and frees
 * nothing on the device (the context, created before, is the caller's).  It
 * needs (2 restart + 4) FP64 vectors of the context's largest finest grid,
 * n (n + 1) values each rounded up to a multiple of 64, plus
 * (restart + 2) (256 + 4) values: for n = 255 and restart = 30, 33.5 MB; for
 * n = 1023, restart <= 2.  Larger requests return MG_ERR_ARG before any work.
 * Every call on one GPU uses that GPU's one array and leaves its contents
 * behind (nothing in it is read before this call writes it): calls that
 * overlap on one GPU - two streams, two threads, two contexts - race.
 * Arguments, outputs, errors and synchronisation as mg_solve_fgmres. */
#define MG_FGMRES_NOALLOC_BYTES (64ll << 20)
mg_status mg_solve_fgmres_noalloc(mg_ctx ctx, const double *const *f, double *const *u, double rtol,
                                  int32_t maxit, int32_t restart, int32_t *iters, double *relres, int32_t *status,
                                  double *history);

/* Per problem: 1 if the last mg_solve switched it from the learned smoother
 * to damped Jacobi (mg_options.fallback), else 0.  flags: host [nprob]. */
mg_status mg_last_fallbacks(mg_ctx ctx, int32_t *flags);

/* Time of the last mg_solve's device work in milliseconds (HIP events). */
mg_status mg_last_solve_ms(mg_ctx ctx, double *ms);

/* Kernel timing for roofline reports: launches each solver kernel on the
 * finest level of problem 0 (the whole size class of that level; the bottom-
 * levels kernel on every problem), reps times back to back between HIP events
 * on the library's stream, and writes the mean duration per launch in
 * milliseconds to ms[0 .. MG_NUM_TIMED_KERNELS-1] (kernel k is named by
 * mg_kernel_name(k)).  V(1,1) solves use outer_residual, check, descend,
 * ascend and bottom; other sweep counts use the step-by-step kernels.
 * Leaves the context's vectors undefined (the next mg_solve resets them).
 * Synchronises. */
#define MG_NUM_TIMED_KERNELS 11
mg_status mg_time_kernels(mg_ctx ctx, int32_t reps, double *ms);
const char *mg_kernel_name(int32_t k);

/* Workgroup shapes of the fused V(1,1) level kernels (kernel 0: descent,
 * 1: ascent), chosen per level size for the batched size classes.  Every
 * shape computes each node with the same arithmetic in the same order, so
 * the choice changes speed only, never results.
 *
 * mg_autotune times each of the MG_NUM_TILES shapes of both kernels on every
 * level size above the bottom kernel's (reps launches after one warm-up, on
 * the context's own buffers and batch) and keeps the fastest.  cache: NULL,
 * or the path of a text file of "key = shape" lines: choices found there are
 * taken without timing, new ones are appended (the file is rewritten);
 * MG_ERR_ARG if it cannot be written.  Contexts whose sweeps are not V(1,1)
 * have nothing to tune (MG_OK).  Leaves the context's vectors undefined (the
 * next mg_solve resets them).  Synchronises. */
#define MG_NUM_TILES 9
mg_status mg_autotune(mg_ctx ctx, int32_t reps, const char *cache);
/* The shape in use for kernel on level size n, and (ms non-NULL) the time per
 * launch of each shape at the last mg_autotune (MG_NUM_TILES entries, 0 when
 * not timed).  MG_ERR_ARG if no level of size n runs the fused kernels. */
mg_status mg_get_tile(mg_ctx ctx, int32_t kernel, int32_t n, int32_t *tile, double *ms);
/* Forces a shape for kernel on level size n (n = 0: every size). */
mg_status mg_set_tile(mg_ctx ctx, int32_t kernel, int32_t n, int32_t tile);
/* Static description of a shape ("32x8 coarse nodes, 512 threads"). */
const char *mg_tile_name(int32_t kernel, int32_t tile);

/* ------------------------------------------------------------------------ */
/* Smoother network (section 4.2, convolutional parameterisation).           */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t nlayers;         /* must be 4                                   */
    const int32_t *channels; /* must be {9, 32, 32, 32, 25}                 */
} mg_net_desc;

/* Creates a network with all parameters zero (the smoother is then damped
 * Jacobi: W = omega * delta_0) and zero Adam state. */
mg_status mg_net_create(const mg_net_desc *d, void *stream, mg_net *out);
mg_status mg_net_destroy(mg_net net);
mg_status mg_net_num_params(mg_net net, int64_t *np);

/* Parameters as a host FP32 vector: per layer, weights [Cout][Cin][3][3]
 * (cross-correlation, ky = row offset + 1, kx = column offset + 1) then bias
 * [Cout].  mg_net_set also clears the optimiser state.  Both synchronise. */
mg_status mg_net_get(mg_net net, float *host, int64_t len);
mg_status mg_net_set(mg_net net, const float *host, int64_t len);

/* Checkpoint: parameters, Adam moments and step count in a little-endian
 * binary file with a versioned header.  Synchronises. */
mg_status mg_net_save(mg_net net, const char *path);
mg_status mg_net_load(mg_net net, const char *path);

/* One training step on the high-frequency smoothing loss
 *   L = 1/(B J) sum_b sum_j || v_bj - H_b A_b v_bj ||_2,
 * H_b the smoother the network produces from stencil A_b (section 3.1: the
 * smoother has to remove only the errors the coarse grid cannot, and by the
 * paper's Theorem 3 the mean of ||X z|| over random unit vectors z tracks
 * ||X||_F), followed by an Adam update of the parameters. */
typedef struct {
    int32_t nprob;               /* B */
    const int32_t *n;            /* host [B] grid sizes (odd, 3..255)                        */
    const double *const *stencil;/* host [B] device pointers, [9][n_b][n_b] FP64             */
    const float *const *vectors; /* host [B] device pointers, [nvec][n_b][n_b] FP32 unit vectors */
    int32_t nvec;                /* J >= 1                                                    */
} mg_train_batch;

typedef struct {
    float lr, beta1, beta2, adam_eps; /* Adam (defaults 1e-3, 0.9, 0.999, 1e-8)            */
    double omega;                     /* 2/3                                                */
    int32_t precision;                /* 0: FP32 forward/backward (parity); 1: BF16 on MFMA  */
    int32_t apply_update;             /* 0: loss and gradient only                         */
} mg_train_opts;

void mg_train_opts_default(mg_train_opts *o);

/* loss (host, may be NULL) receives L; grad (host [num_params], may be NULL)
 * receives dL/dparams.  Synchronises when either is requested. */
mg_status mg_train_step(mg_net net, const mg_train_batch *b, const mg_train_opts *o, float *loss,
                        float *grad);

/* The same training step on problems the library draws up itself: for every
 * problem b the Q1 stencil of the rotated tensor (theta[b], eps[b]) on an
 * n[b] x n[b] grid (as mg_stencil_q1_rotated) and nvec high-frequency vectors
 * taken from the pool of its grid size at index[b * nvec + j].  Steps of the
 * same structure (nprob, n, nvec, the pools, the options) replay one captured
 * HIP graph holding every launch of the step - stencils, vector gather,
 * forward, loss, backward, Adam - with the per-step tensors, indices and the
 * Adam step number uploaded just before the replay; a different structure
 * rebuilds it (and the first call allocates).  The network's later eager
 * calls do not disturb it.  Adam's bias corrections are computed on the
 * device (FP64 pow), which may differ from mg_train_step's host values in the
 * last bit.  Pools stay the caller's and must not change address or size
 * between replays of one structure (pass them again: a change rebuilds). */
typedef struct {
    int32_t nprob;               /* B */
    const int32_t *n;            /* host [B] grid sizes (odd, 3..255) */
    const double *theta;         /* host [B] */
    const double *eps;           /* host [B], 0 < eps <= 1 */
    int32_t npools;
    const int32_t *pool_n;       /* host [npools]: the grid size of each pool */
    const float *const *pool;    /* host [npools] device pointers, [pool_size][pool_n][pool_n] FP32 unit vectors */
    const int32_t *pool_size;    /* host [npools] */
    const int32_t *index;        /* host [B][nvec]: pool entries per problem */
    int32_t nvec;                /* J >= 1 */
} mg_train_draw;

mg_status mg_train_step_draw(mg_net net, const mg_train_draw *d, const mg_train_opts *o, float *loss, float *grad);

/* ------------------------------------------------------------------------ */
/* Adaptive training (section 3.3, Algorithm 2).                              */
/* ------------------------------------------------------------------------ */

/* The field of the transposed smoother: for the smoother H = W / a_C of
 * stencil A, WT with (WT / a_C) = H^T, i.e.
 *   WT_p[k] = a_C(p) W_{p+off(k)}[24-k] / a_C(p+off(k))  (0 where p+off(k) is
 * off the grid).  A: device [9][n][n], W, WT: device [25][n][n] FP64, W != WT. */
mg_status mg_smoother_transpose(int32_t n, const double *A, const double *W, double *WT, void *stream);

typedef struct {
    int32_t nprob;                /* B: the number of problems of the contexts             */
    const int32_t *k;             /* host [B]: cycles k_b of the loss, 1..64               */
    const double *const *f;       /* host [B] device pointers, [n][n] FP64 right-hand sides */
    const double *const *u0;      /* host [B] device pointers, [n][n] FP64 initial guesses  */
    const double *const *u_star;  /* host [B] device pointers, [n][n] FP64 exact solutions  */
    double *const *dW;            /* NULL, or host [B] device pointers, [25][n][n] FP64,
                                     receiving dL/dW_b (FP64) */
} mg_alpha_batch;

/* One step of the adaptive training of the network on the finest level of
 * the contexts (Algorithm 2): the loss
 *   L = (1/B) sum_b || Phi(u0_b, f_b, k_b) - u*_b ||_2,
 * Phi being k_b cycles of pre-smoothing with the network's smoother H (FP64
 * inference from the current parameters), coarse correction P Psi_c R with
 * one cycle Psi_c of the fixed coarser hierarchy, and post-smoothing with H;
 * the gradient dL/dparams by the adjoint of those cycles (FP64 down to dL/dW,
 * then the network backward in FP32); and an Adam update if o->apply_update.
 * top: FP64 context whose problems all have the same n > coarsest_n; its
 *   finest-level smoother is overwritten by the network's.
 * coarse: FP64 context of the level-1 stencils of top's problems (same order,
 *   mg_get_stencil(top, b, 1)), same coarsest_n, nu_pre == nu_post, with the
 *   fixed smoothers installed (mg_smoother_infer_size / mg_set_smoother, or
 *   damped Jacobi).  Its cycle is Psi_c.
 * coarse_t: like coarse with every smoother transposed (mg_smoother_transpose),
 *   so that its cycle is Psi_c^T; may be coarse itself when coarse's smoothers
 *   are symmetric (damped Jacobi).
 * o: precision must be 0; o->omega is not used (the network output's Jacobi
 *   term takes top's mg_options.omega).
 * Outputs (host, each may be NULL): loss, losses[B] (the unscaled norms),
 * grad[num_params] (dL/dparams).  Runs on top's stream; leaves the coarse
 * contexts' vectors undefined.  MG_ERR_DIVERGED (parameters unchanged) if a
 * norm is not finite.  Synchronises. */
mg_status mg_alpha_step(mg_ctx top, mg_ctx coarse, mg_ctx coarse_t, mg_net net, const mg_alpha_batch *b,
                        const mg_train_opts *o, double *loss, double *losses, float *grad);

/* ---------------------------------------------- convolution-stack smoother
 * The constant-coefficient alpha-CNN smoother of section 5 (full coarsening):
 *     H x = f5(f4(f3(f2(f1(x))))) + f6(x),
 * each f_i a single-channel 3x3 cross-correlation with zero padding (every
 * intermediate grid is zero outside the n x n interior).  Weights: 54 FP64
 * values [6][3][3] (layer, ky, kx), layers 0..4 = f1..f5, layer 5 = f6; tap
 * (ky, kx) multiplies x at (j + ky - 1, i + kx - 1).  H is linear; it is
 * applied to the residual as e += H (r - A e).  The paper initialises f1..f5
 * with zeros and f6 as the Jacobi stencil; with all five composed kernels
 * zero none of them receives a gradient, so the library leaves the
 * initialisation to the caller (mg_inputs.stack_init: f1..f4 random, f5
 * zero). */

/* Installs one level's stack smoother on a context created with
 * MG_SMOOTHER_STACK: phi host [54] FP64 (stored in the context's precision),
 * transpose = 1 installs the stack of H^T instead (the kernels turned by 180
 * degrees, f1..f5 in reverse order), as the adjoint context of
 * mg_stack_alpha_step needs.  Every level above the coarsest of every problem
 * needs weights before mg_vcycle / mg_solve / mg_solve_fgmres (MG_ERR_STATE).
 * normalised = 1: phi was made for an operator whose centre entry is 1 (a
 * trained stack is stored that way); f5 and f6, which carry the scale of
 * H ~ 1/a_C, are divided by the mean centre entry of the level's stencil
 * (constant-coefficient operators have one value), so that one set of
 * weights serves every level of a Galerkin hierarchy.  0: phi as given.
 * Synchronises. */
mg_status mg_set_stack(mg_ctx ctx, int32_t prob, int32_t level, const double *phi, int32_t transpose,
                       int32_t normalised);

/* Replaces the stack a level applies after the coarse correction (mg_set_stack
 * installs the same weights before and after, as Algorithm 2 does).  With the
 * level's own weights and transpose = 1, the post-smoother is H^T and the
 * cycle's error propagation is self-adjoint in the A inner product (the
 * symmetric V-cycle): the A-norm of one cycle then equals its spectral radius,
 * so a convergent coarse cycle cannot amplify errors once nested inside a
 * finer one.  normalised as for mg_set_stack.  MG_ERR_STATE before
 * mg_set_stack on that level.  Synchronises. */
mg_status mg_set_stack_post(mg_ctx ctx, int32_t prob, int32_t level, const double *phi, int32_t transpose,
                            int32_t normalised);

/* y_c (+)= H x_c for c < count: x, y device [count][n][n] FP64 (must not
 * overlap), phi device [54] FP64, accumulate 0 (y = H x) or 1 (y += H x);
 * 1 <= n <= 16383, 0 <= count <= 65535 (else MG_ERR_ARG).  Asynchronous on
 * stream. */
mg_status mg_stack_apply(int32_t n, int32_t count, const double *phi, const double *x, double *y,
                         int32_t accumulate, void *stream);

/* One step of the adaptive training of a level's stack smoother (Algorithm
 * 2, section 3.3): for the instances b of top (one problem, B right-hand
 * sides, or several problems of one size), the loss
 *   L = (1/B) sum_b || Phi(u0_b, f_b, k_b) - u*_b ||_2,
 * Phi being k_b cycles of pre-smoothing with H, coarse correction
 * P Psi_c R with one cycle of the fixed coarser hierarchy, post-smoothing
 * with H; its gradient with respect to the 54 weights by the adjoint of
 * those cycles (FP64); and, if o->apply_update, an FP64 Adam step (o's lr,
 * beta1, beta2, adam_eps; t the 1-based step number for the bias correction)
 * on phi with the moments adam_m, adam_v.  symmetric = 1: H^T after the
 * coarse correction on the trained level (the symmetric cycle of
 * mg_set_stack_post); its coarse hierarchy is then symmetric too, and coarse
 * may be passed as coarse_t.
 * top: FP64 context, every problem of the same n > coarsest_n (its smoother
 *   setting is not used).
 * coarse, coarse_t: FP64 contexts of the level-1 stencils of top's problems
 *   (same order), nu_pre == nu_post, with the fixed coarser smoothers
 *   installed; coarse_t with every smoother transposed (mg_set_stack with
 *   transpose = 1; a damped Jacobi or coarsest-only context is its own
 *   transpose and may be passed as both).
 * phi, adam_m, adam_v: device [54] FP64 (phi updated in place).
 * b: as for mg_alpha_step, with dW null.
 * loss: host, the mean loss; losses: host [B] or NULL; grad: host [54] FP64
 *   or NULL, dL/dphi.
 * MG_ERR_DIVERGED (weights unchanged) if a norm is not finite.  Synchronises. */
mg_status mg_stack_alpha_step(mg_ctx top, mg_ctx coarse, mg_ctx coarse_t, double *phi, double *adam_m,
                              double *adam_v, int32_t t, int32_t symmetric, const mg_alpha_batch *b,
                              const mg_train_opts *o, double *loss, double *losses, double *grad);

/* ------------------------------------------------------------------------ */
/* Red-black coarsening (section 6.1) with the two-layer convolution smoother  */
/* H = f2(f1) (section 6, "Neural networks").                                  */
/* ------------------------------------------------------------------------ */

/* Levels alternate between a full grid and its checkerboard: level 0 is the
 * n x n grid; a full N x N level coarsens to the nodes with i + j even of the
 * same array ("black"; a semi-coarsening along the 45-degree direction); a
 * checkerboard level coarsens, on its 45-degree rotated mesh, to the full
 * (N - 1)/2 grid of the nodes with i and j both odd (coarse node I on fine
 * node 2I + 1).  Transfers: restriction (1/8)[0 1 0; 1 4 1; 0 1 0] and
 * interpolation (1/4)][0 1 0; 1 4 1; 0 1 0][ along the level's mesh axes
 * (the grid axes on a full level, the diagonals on a checkerboard); coarse
 * operators Galerkin R A P (their footprints grow to 45 entries); the last
 * level solved directly (at most 49 points).  As the paper pads its irregular
 * grids with zeros, every level's vectors are N x N arrays that are zero off
 * the level's points (values given there are ignored).  Every call is FP64.
 * Smoothers: damped Jacobi (omega = 2/3, default) or
 *   H x = M f2(f1(M x)),
 * f1, f2 single-channel 3x3 cross-correlations on the N x N array with zero
 * padding, M the level's point mask; weights: 18 FP64 [2][3][3] (layer, ky,
 * kx), tap (ky, kx) multiplying x at (j + ky - 1, i + kx - 1). */
typedef struct mg_rb_s *mg_rb;

/* Builds the hierarchy of one operator: stencil device [9][n][n] FP64
 * (conventions above; validated: MG_ERR_ARG), nlevels >= 1 levels in all
 * (the last solved directly: MG_ERR_ARG if it has more than 49 points or the
 * grid is too small), the Galerkin levels and the last level's inverse on the
 * device.  n = 2^k - 1 <= 8191.  Synchronises. */
mg_status mg_rb_create(int32_t n, const double *stencil, int32_t nlevels, void *stream, mg_rb *out);
mg_status mg_rb_destroy(mg_rb h);
/* Level shape: N (array side), checker (0 full, 1 checkerboard), noffsets (stencil footprint). */
mg_status mg_rb_level(mg_rb h, int32_t level, int32_t *N, int32_t *checker, int32_t *noffsets);
/* The level's operator: offsets host [2 K] (dx, dy pairs; may be NULL) and its field, out device
 * [K][N][N] (may be NULL): row (i, j) couples to (i + dx_c, j + dy_c) with out[c][j][i]. */
mg_status mg_rb_get_stencil(mg_rb h, int32_t level, int32_t *offsets, double *out);
/* Installs the two-layer smoother on a level above the last: phi host [18], or NULL for damped
 * Jacobi.  a_ref > 0: the weights were made for an operator whose centre entry is a_ref; f1 is
 * taken times a_ref / a_C, a_C the level's centre entry at its middle node (N/2, N/2), so that H
 * keeps its scale relative to the operator (a_ref = 0: as given).  Synchronises. */
mg_status mg_rb_set_smoother(mg_rb h, int32_t level, const double *phi, double a_ref);
/* e = V(r) from `level` down (Algorithm 1 in correction form, nu_pre / nu_post sweeps in [0, 8])
 * for nvec vectors: r, e device [nvec][N][N] of that level. */
mg_status mg_rb_vcycle(mg_rb h, int32_t level, int32_t nvec, const double *r, double *e, int32_t nu_pre,
                       int32_t nu_post);
/* The stationary solve u_0 = 0, u += V(f - A u) until ||f - A u|| <= rtol ||f|| (section 6.1
 * stopping rule) or maxit cycles, on `level`'s operator (0: the input grid) with the levels below
 * it, for nvec right-hand sides f (device [nvec][N][N] of that level); u receives the solutions.
 * Host outputs as in mg_solve (each may be NULL; history [nvec][maxit + 1]).  Synchronises. */
mg_status mg_rb_solve(mg_rb h, int32_t level, int32_t nvec, const double *f, double *u, double rtol,
                      int32_t maxit, int32_t nu_pre, int32_t nu_post, int32_t *iters, double *relres,
                      int32_t *status, double *history);
/* Device time of the last mg_rb_solve in milliseconds. */
mg_status mg_rb_last_solve_ms(mg_rb h, double *ms);
/* One step of the adaptive training (Algorithm 2) of `level`'s two-layer smoother: for B
 * instances (f, u0, u_star device [B][N][N] of that level, k host [B] in [1, 64]) the loss
 *   L = (1/B) sum_b || Phi(u0_b, f_b, k_b) - u*_b ||_2,
 * Phi being k_b cycles of: pre-smoothing with H (weights phi, device [18]), coarse correction
 * P Psi_c R with one V(1,1) cycle Psi_c of the levels below (their installed smoothers),
 * post-smoothing with H; its gradient with respect to the 18 weights (forward mode: each instance
 * runs with its 18 tangents), and an Adam step (o->lr, beta1, beta2, adam_eps; step t >= 1) on
 * phi with the moments adam_m, adam_v (device [18]) if o->apply_update (o NULL: the defaults).
 * loss: host; losses: host [B] or NULL; grad: host [18] or NULL.  B * 19 <= 65535.
 * MG_ERR_DIVERGED (weights unchanged) if the loss is not finite.  Synchronises. */
mg_status mg_rb_alpha_step(mg_rb h, int32_t level, double *phi, double *adam_m, double *adam_v, int32_t t,
                           int32_t B, const int32_t *k, const double *f, const double *u0, const double *u_star,
                           const mg_train_opts *o, double *loss, double *losses, double *grad);

/* ------------------------------------------------------------------------ */
const char *mg_status_str(mg_status s);
const char *mg_last_error(void);
/* Library version string. */
const char *mg_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MGCNN_H */
