// Red-black coarsening (section 6.1) and its two-layer convolution smoother
// H = f2(f1) (section 6, "Neural networks"): kernels and their launchers.
//
// Levels alternate between a full N x N grid and its checkerboard (the nodes
// with i + j even), which is stored padded on the same N x N array with zeros
// on the other nodes, as the paper pads the irregular grids for its networks.
// A checkerboard level coarsens to the full grid of the nodes with i, j both
// odd (size (N - 1)/2, node I on fine node 2I + 1).  Every level vector has
// rows of pitch P = N + 1; a batch of vectors sits at a stride of N * P.
#pragma once
#include "common.hpp"

namespace mg {

constexpr int kRBMaxOffsets = 48;      // Galerkin footprints reach 45 entries (full: 7x7 less the
                                       // corners; checkerboard: the even offsets within |d| <= 5)
constexpr int kRBMaxLevels = 28;
constexpr int kRBMaxCoarse = 49;       // unknowns of the directly solved last level
constexpr int kRBWeights = 18;         // [2][3][3]: f1, f2
enum { kRBFull = 0, kRBChecker = 1 };

// A level's stencil footprint: offset c couples node (i, j) to (i + dx[c], j + dy[c]); kc is the
// index of (0, 0).  Passed to kernels by value.
struct RBOffsets {
    int K, kc;
    int8_t dx[kRBMaxOffsets], dy[kRBMaxOffsets];
};

struct RBGeom {
    int N, P, kind;
    int64_t vs;  // vector stride of a batch (N * P)
};

// The level's point set.
__host__ __device__ inline bool rb_has(int kind, int i, int j) { return kind == kRBFull || ((i + j) & 1) == 0; }

// y_v = (b_v) + sign * A x_v on the level's points, zero elsewhere; b may be null (then y = sign A x).
// active: per-vector flags or null.
void launch_rb_residual(const RBGeom &g, const RBOffsets &o, const double *A, const double *b, const double *x,
                        double *y, double sign, int nvec, const int *active, hipStream_t st);
// r_v = f_v - A u_v and the block sums of r_v^2 into partial[v][rb_norm_blocks(N)].
int rb_norm_blocks(int N);
void launch_rb_outer(const RBGeom &g, const RBOffsets &o, const double *A, const double *f, const double *u,
                     double *r, double *partial, int nvec, const int *active, hipStream_t st);
// out[v] = sum of partial[v][*] (fixed order).
void launch_rb_sum(const double *partial, int nb, double *out, int nvec, hipStream_t st);
// e_v (+)= omega s_v / a_C on the level's points.
void launch_rb_jacobi(const RBGeom &g, const double *Acentre, double omega, const double *s, double *e,
                      bool accumulate, int nvec, const int *active, hipStream_t st);
// y_v (+)= Mout conv3(Min x_v, w) with w device [9] (zero padding on the N x N array); mask_in /
// mask_out: apply the level's point mask to the input / output (else the whole array).
void launch_rb_conv(const RBGeom &g, const double *w, const double *x, double *y, bool mask_in, bool mask_out,
                    bool accumulate, int nvec, const int *active, hipStream_t st);
// The derivative of H x_v with respect to each of the 18 weights, added to dy[v][j] (tangent j of
// instance v at stride vs, tangent stride tstride): layer-1 tap k: M f2(unit_k(M x)); layer-2 tap
// k: M unit_k(t) with t = f1(M x) (given).  w: device [18].
void launch_rb_dH(const RBGeom &g, const double *w, const double *x, int64_t xstride, const double *t,
                  int64_t tstride_t, double *dy, int64_t ystride, int64_t tstride, int ninst, const int *active,
                  int active_stride, hipStream_t st);
// rc_v = R s_v from the fine level gf to its coarse level gc.
void launch_rb_restrict(const RBGeom &gf, const RBGeom &gc, const double *s, double *rc, int nvec,
                        const int *active, hipStream_t st);
// e_v += P ec_v.
void launch_rb_prolong(const RBGeom &gf, const RBGeom &gc, const double *ec, double *e, int nvec, const int *active,
                       hipStream_t st);
// Galerkin: Ac = R Af P on the coarse level's footprint.
void launch_rb_galerkin(const RBGeom &gf, const RBOffsets &of, const double *Af, const RBGeom &gc,
                        const RBOffsets &oc, double *Ac, hipStream_t st);
// Dense inverse of the last level's operator on its m points (Cholesky in LDS); flag |= 8 if not SPD.
void launch_rb_coarse_factor(const RBGeom &g, const RBOffsets &o, const double *A, int m, double *Ainv, int *flag,
                             hipStream_t st);
// e_v = Ainv r_v on the last level's points.
void launch_rb_coarse_apply(const RBGeom &g, int m, const double *Ainv, const double *r, double *e, int nvec,
                            const int *active, hipStream_t st);
// Level 0's nine-point field (pitched): flag |= 2 if a centre entry is not positive, 1 if an entry
// coupling off the grid is nonzero (or any entry is not finite).
void launch_rb_validate(const RBGeom &g, const double *A, int *flag, hipStream_t st);
// Copies between dense [v][N][N] arrays and pitched level vectors (masked: zero off the level's points);
// destination vectors dstride elements apart.
void launch_rb_copy_in(const RBGeom &g, const double *src, double *dst, int64_t dstride, int nvec, hipStream_t st);
void launch_rb_copy_out(const RBGeom &g, const double *src, double *dst, int nvec, hipStream_t st);
// y_v += x_v (level points).
void launch_rb_axpy(const RBGeom &g, const double *x, double *y, int nvec, const int *active, hipStream_t st);
// Per instance b (vector b * stride): out[b][0] = ||x_b - y_b||^2 block sums, out[b][1 + j] = block sums of
// <tangent j, x_b - y_b> (tangent j at x_b + (1 + j) * vs); partial layout [b][19][nb].
void launch_rb_alpha_dots(const RBGeom &g, const double *u, int64_t inst_stride, const double *ustar,
                          double *partial, int ninst, const int *want, hipStream_t st);
// Per-vector solver state of a red-black solve.
struct RBState {
    int active, iters, status, pad;  // status: 0 running / converged, 1 not converged, -4 diverged
    double fnorm, relres;
};
// The stopping rule from rr[v] = ||f_v - A u_v||^2 (init: rr = ||f||^2, set up the state); act[v]
// mirrors state[v].active for the cycle kernels; history[v][iters] (or null) records relres.
void launch_rb_check(const double *rr, RBState *state, int *act, double tol, int maxit, double *history,
                     int hist_stride, int init, int nvec, hipStream_t st);
// From sums[b][19] (||d_b||^2, <tangent_j, d_b>): out[0] = mean_b ||d_b||, out[1 + b] = ||d_b||,
// out[1 + B + j] = mean_b <tangent_j, d_b> / ||d_b|| (the loss gradient).
void launch_rb_alpha_final(const double *sums, int B, double *out, hipStream_t st);
// Adam on n FP64 parameters (step t >= 1).
void launch_rb_adam(int n, double *w, double *m, double *v, const double *g, int t, double lr, double b1, double b2,
                    double eps, hipStream_t st);

}  // namespace mg
