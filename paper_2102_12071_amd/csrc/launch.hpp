// Host-side launchers of the device kernels (one translation unit per kernel
// family; the host runtime calls only these).
#pragma once
#include "common.hpp"

namespace mg {

// ---- stencil.hip: discretisation and coarsening (FP64) ----
void launch_q1_rotated(int n, int P, int64_t plane, double theta, double eps, double *out, hipStream_t st);
// K = R(theta) diag(1, eps) R(theta)^T: k = {k11, k12, k22}.
void q1_tensor(double theta, double eps, double *k);
// Q1 stencils of count problems of size n, tensors k (device [count][3]); out: [count][9][n][n].
void launch_q1_rotated_batch(int n, int count, const double *k, double *out, hipStream_t st);
void launch_cellavg5(int n, const double *a, int Pa, int P, int64_t plane, double *out, hipStream_t st);
void launch_galerkin(int n, int P, int64_t plane, const double *A, int Pc, int64_t planec, double *Ac,
                     hipStream_t st);
void launch_copy_field(int n, int nch, const double *src, int Ps, int64_t planes, double *dst, int Pd,
                       int64_t planed, hipStream_t st);
void launch_to_f32(int64_t count, const double *src, float *dst, hipStream_t st);
void launch_validate(int n, int P, int64_t plane, const double *A, int *flag, hipStream_t st);
// Level 0 from the caller's dense [9][n][n] stencil in one pass: pitched FP64 copy, FP32 copy (A32 not
// null), the checks of launch_validate into *flag, and the symmetry flags of launch_check_symmetric for
// the FP64 entries (*sym64) and for the entries the cycle reads (*symc: FP32 when A32 is given).
void launch_ingest(int n, const double *src, int P, int64_t plane, double *A64, float *A32, int *flag, int *sym64,
                   int *symc, hipStream_t st);
// *sym = 1 if A[c](p) == A[8-c](p + d_c) for c < 4 wherever both nodes are on the grid, else 0.
template <typename T>
void launch_check_symmetric(int n, int P, int64_t plane, const T *A, int *sym, hipStream_t st);
// Dirichlet nodes of a domain mask (0 = outside) on a dense [9][n][n] stencil; out may alias A.
void launch_mask(int n, const uint8_t *mask, const double *A, double *out, hipStream_t st);

// ---- coarse.hip: coarsest-level factorisation (explicit inverse) ----
void launch_coarse_factor(int m, int P, int64_t plane, const double *A, double *Ainv, int *flag, hipStream_t st);

// ---- fused.hip: one launch per level and direction for V(1,1) ----
// tile: one of kNumTiles workgroup shapes (0 = default); results do not depend on it.
constexpr int kNumTiles = 9;
template <typename T>
void launch_descend(const CycleSlot<T> *slots, int nslots, int n, bool cnn, double omega, const SolveState *state,
                    hipStream_t st, int tile = 0);
template <typename T>
void launch_ascend(const CycleSlot<T> *slots, int nslots, int n, bool cnn, double omega, const SolveState *state,
                   hipStream_t st, int tile = 0);
// "32x8 coarse nodes, 512 threads" and the like (kernel 0: descent, 1: ascent).
const char *tile_name(int kernel, int tile);

// ---- krylov.hip: FP64 vectors of the flexible-GMRES solver (finest grid, pitch P) ----
constexpr int kKrylovBlocks = 256;  // partial sums per dot product
// the fixed workspace of mg_solve_fgmres_noalloc: bytes per GPU, and its device address on the
// current device (looked up once per device)
constexpr size_t kKrylovStaticBytes = size_t(64) << 20;
hipError_t krylov_static_workspace(double **ptr);
// y = b + sign * A x (b may be null)
void launch_kr_apply(int n, int P, int64_t plane, const double *A, const double *x, const double *b, double sign,
                     double *y, hipStream_t st);
// out[v] = <w, V_v> for v < nv (V_v = V + v * vstride), or sqrt of it when root; partial: nv * kKrylovBlocks
void launch_kr_dots(int n, int P, const double *w, const double *V, int64_t vstride, int nv, double *partial,
                    double *out, int root, hipStream_t st);
// w -= sum_v coef[v] V_v (coef on the device)
void launch_kr_update(int n, int P, double *w, const double *V, int64_t vstride, int nv, const double *coef,
                      hipStream_t st);
// y = x / *d
void launch_kr_scale(int n, int P, const double *x, const double *d, double *y, hipStream_t st);
// u += sum_k coef[k] Z_k
void launch_kr_combine(int n, int P, double *u, const double *Z, int64_t vstride, int nz, const double *coef,
                       hipStream_t st);

// ---- cycle.hip: V-cycle kernels (T = float: mixed precision; double: FP64) ----
// Every launcher covers one size class (all slots share n); blocks of
// problems that are no longer active return at once.
template <typename T>
void launch_outer_residual(const OuterSlot<T> *slots, int nslots, int n, const SolveState *state, hipStream_t st);
// Number of partial sums launch_outer_residual writes per slot for size n.
int outer_residual_parts(int n);
template <typename T>
void launch_check(const OuterSlot<T> *slots, int nslots, SolveState *state, const SolveParams *prm, int init,
                  hipStream_t st);
// Marks every problem active (single-cycle use, and before the first residual).
void launch_activate(SolveState *state, int nprob, hipStream_t st);
// Sets a level vector to zero (FP64 state at the start of a solve).
void launch_zero_f64(double *x, int64_t count, hipStream_t st);
template <typename T>
void launch_update_u(const OuterSlot<T> *slots, int nslots, int n, const SolveState *state, hipStream_t st);
template <typename T>
void launch_smooth_first(const CycleSlot<T> *slots, int nslots, int n, bool cnn, double omega,
                         const SolveState *state, hipStream_t st);
template <typename T>
void launch_residual(const CycleSlot<T> *slots, int nslots, int n, const SolveState *state, hipStream_t st);
template <typename T>
void launch_smooth_apply(const CycleSlot<T> *slots, int nslots, int n, bool cnn, double omega,
                         const SolveState *state, hipStream_t st);
template <typename T>
void launch_residual_restrict(const CycleSlot<T> *slots, int nslots, int n, const SolveState *state,
                              hipStream_t st);
template <typename T>
void launch_prolong(const CycleSlot<T> *slots, int nslots, int n, const SolveState *state, hipStream_t st);
template <typename T>
void launch_zero_e(const CycleSlot<T> *slots, int nslots, int n, const SolveState *state, hipStream_t st);

// ---- bottom.hip: all levels with n <= kBottomMax, one workgroup per problem ----
template <typename T>
size_t bottom_smem_bytes(int top_n);
template <typename T>
// prm: also apply the solver's stopping rule to the outer residual's block sums (null: the cycle only).
void launch_bottom(const BottomSlot<T> *slots, int nslots, int top_n, bool cnn, double omega, int nu1, int nu2,
                   SolveState *state, const SolveParams *prm, hipStream_t st);
template <typename T>
void prepare_bottom();

// ---- cnn.hip: smoother inference ----
// Direct (VALU) 3x3 convolution layer, "same" zero padding; planes of pitch P.
template <typename T>
void launch_cnn_input(int n, int P, int64_t plane, const T *A, T *x0, hipStream_t st);
template <typename T>
void launch_conv3x3_direct(int n, int P, int64_t plane, int cin, int cout, const T *w, const T *b, const T *in,
                           T *out, bool relu, hipStream_t st);
template <typename T>
void launch_cnn_output(int n, int P, int64_t plane, const T *A, const T *y, double omega,
                       typename SmootherStore<T>::type *H, hipStream_t st);
void launch_f32_to_f64(int64_t count, const float *src, double *dst, hipStream_t st);
// Fused four-layer BF16 MFMA inference (9 -> 32 -> 32 -> 32 -> 25) writing
// H = W / a_C in BF16.  packed: weights laid out by launch_pack_weights_mfma
// into a buffer of packed_net_bytes().
size_t packed_net_bytes();
void launch_pack_weights_mfma(const float *params, void *packed, hipStream_t st);
// One level of the one-launch smoother inference: its tiles are blocks
// [tile0, tile0 + cnn_level_tiles(n)) of the launch.
struct CnnLevelDesc {
    int n, P;
    int64_t plane;
    const float MG_G *A32;  // 9 planes FP32
    bf16_t MG_G *H;         // 25 planes BF16 out
    int tile0;
};

// Packed networks by level size, for one inference launch over levels that take different networks.
constexpr int kMaxNetSizes = 16;
struct CnnNetMap {
    int count;                       // 0: every level takes the launch's single network
    int n[kMaxNetSizes];             // level size
    const void *packed[kMaxNetSizes];  // its network (packed_net_bytes() each, device)
};

// One launch over the levels of desc (device, tile0 ascending; size_filter != 0: only levels of that size).
// map.count > 0: a level of size map.n[k] takes map.packed[k] (every level's size must be listed).
int cnn_level_tiles(int n);
void launch_cnn_fused_levels(const CnnLevelDesc *desc, int ndesc, int total_tiles, int size_filter, const void *packed,
                             const CnnNetMap &map, double omega, hipStream_t st);
// Smoother field conversions for mg_set_smoother / mg_get_smoother.
// H = W / a_C (a_C from the FP64 stencil), and back.
template <typename T>
void launch_set_smoother(int n, int P, int64_t plane, const double *W, int Pw, int64_t planew, const double *A64,
                         typename SmootherStore<T>::type *H, hipStream_t st);
// Damped Jacobi written as the smoother field (H = omega / a_C at the centre tap).
template <typename T>
void launch_jacobi_smoother(int n, int P, int64_t plane, const double *A64, double omega,
                            typename SmootherStore<T>::type *H, hipStream_t st);
template <typename T>
void launch_get_smoother(int n, int P, int64_t plane, const typename SmootherStore<T>::type *H,
                         const double *A64, double *W, int Pw, int64_t planew, hipStream_t st);

}  // namespace mg
