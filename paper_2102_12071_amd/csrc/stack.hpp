// Convolution-stack smoother (the constant-coefficient alpha-CNN of section 5,
// full coarsening): kernels and their launchers.
#pragma once
#include "common.hpp"

namespace mg {

constexpr int kStackWeights = 54;  // [6][3][3]: f1..f5 composed, then f6

// The smoothing sweeps of the step-by-step cycle with the stack smoother: the
// slot's H points to the level's two weight sets of 54 (type T), before and
// after the coarse correction.  mode 0: e = H r (first sweep); 1: e += H s
// (s = r - A e from the residual kernel); 2: e += H' s with the second set.
enum { kStackFirst = 0, kStackPre = 1, kStackPost = 2 };
template <typename T>
void launch_stack_cycle(const CycleSlot<T> *slots, int nslots, int n, int mode, const SolveState *state,
                        hipStream_t st);

// Fused V(1,1) level kernels with the stack smoother (levels with n > kBottomMax):
// descend (e = H r, s = r - A e, r_c = R s; nc = the coarse size) and ascend
// (e' = e + P e_c, s = r - A e', e = e' + H' s into u on the finest level, into s
// on the others, which the next finer ascent reads as e_c).
template <typename T>
void launch_stack_descend(const CycleSlot<T> *slots, int nslots, int nc, const SolveState *state, hipStream_t st);
template <typename T>
void launch_stack_ascend(const CycleSlot<T> *slots, int nslots, int n, const SolveState *state, hipStream_t st);

// All levels with n <= kBottomMax of every problem in one workgroup each
// (bottom slots whose H points to each level's two weight sets); the top
// level's r in, its e out.  prepare_stack_bottom once per compute type before.
template <typename T>
void prepare_stack_bottom();
template <typename T>
// prm: also apply the solver's stopping rule to the outer residual's block sums (null: the cycle only).
void launch_stack_bottom(const BottomSlot<T> *slots, int nslots, int top_n, int nu1, int nu2, SolveState *state,
                         const SolveParams *prm, hipStream_t st);

// y_z (+)= H x_z for z < count, vectors of pitch P at stride vs, one weight
// set w (device, [54]); active (or null) skips vectors.  x and y must not overlap.
void launch_stack_vecs(const double *x, double *y, int64_t vs, const double *w, int n, int P, int count,
                       bool accumulate, const int *active, hipStream_t st);

// y_z = C x_z for the single layer with kernel w[9] (turned by 180 degrees
// when flip: the transposed correlation).
void launch_stack_layer(const double *x, double *y, int64_t vs, const double *w, bool flip, int n, int P, int count,
                        const int *active, hipStream_t st);

// The gradient of <g, H x> with respect to the 54 weights, per layer L the
// correlation of g[L] with x[L] over the grid, added into part[z][block][54].
struct StackPairs {
    const double *g[6];
    const double *x[6];
};
int stack_wgrad_blocks(int n);
void launch_stack_wgrad(const StackPairs &pr, int64_t vs, int n, int P, int count, const int *active, double *part,
                        hipStream_t st);
// grad[54] = sum over the rows of part ([nrow][54]), in row order.
void launch_stack_gsum(const double *part, int64_t nrow, double *grad, hipStream_t st);
// The weights of H^T.
void launch_stack_transpose(const double *w, double *wT, hipStream_t st);
// out[0] = the mean centre entry of a level's FP64 stencil (device).
void launch_stack_mean_centre(int n, int P, int64_t plane, const double *A, double *out, hipStream_t st);
// Adam on the 54 weights (FP64), step t >= 1.
void launch_stack_adam(double *w, double *m, double *v, const double *g, int t, double lr, double b1, double b2,
                       double eps, hipStream_t st);

}  // namespace mg
