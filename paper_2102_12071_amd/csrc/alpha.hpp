// Kernels of the adaptive training step (Algorithm 2), FP64.
#pragma once
#include "common.hpp"

namespace mg {

// One problem of a training stage: the trained level (pitch P) and the
// finest-level buffers of the two coarse contexts (which = 0: the fixed
// coarse cycle, 1: the same cycle with every smoother transposed; pitch nc + 1).
struct AlphaProb {
    const double MG_G *A;   // [9] planes, stencil of the trained level
    const double MG_G *H;   // [25] planes, its smoother H = W / a_C
    double MG_G *rc[2];     // coarse right-hand side
    double MG_G *uc[2];     // coarse solution (cleared with each restriction; the cycle adds its correction)
};

// Level vectors: problem z at offset z * vs (pitch P); active[z] = 0 skips a problem.
void launch_al_apply_A(const AlphaProb *pr, int nb, int n, int P, int64_t plane, int64_t vs, const double *x,
                       const double *b, double sign, double *y, const int *active, hipStream_t st);
void launch_al_H(const AlphaProb *pr, int nb, int n, int P, int64_t plane, int64_t vs, const double *x, double *y,
                 bool transpose, bool accumulate, const int *active, hipStream_t st);
void launch_al_outer(int nb, int n, int P, int64_t plane, int64_t vs, const double *g, const double *x, double *dH,
                     const int *active, hipStream_t st);
void launch_al_restrict(const AlphaProb *pr, int which, int nb, int n, int P, int64_t vs, const double *x,
                        const int *active, hipStream_t st);
void launch_al_prolong(const AlphaProb *pr, int which, int nb, int n, int P, int64_t vs, const double *x, double *y,
                       const int *active, hipStream_t st);
void launch_al_axpy(int nb, int n, int P, int64_t vs, const double *x, double s, const double *w, double *y,
                    const int *active, hipStream_t st);
void launch_al_dist(int nb, int n, int P, int64_t vs, const double *x, const double *y, double *dist, hipStream_t st);
void launch_al_seed(int nb, int n, int P, int64_t plane, int64_t vs, const double *x, const double *y,
                    const double *dist, double scale, double *lam, double *dH, hipStream_t st);
void launch_al_dw(const AlphaProb *pr, int nb, int n, int P, int64_t plane, const double *dH, double *const *W64,
                  float *out, hipStream_t st);
// Dense [25][n][n] field W of stencil A to the field of the transposed smoother.
void launch_al_transpose(int n, const double *A, const double *W, double *WT, hipStream_t st);

// Sub-allocation of a step's workspace in 256-byte aligned pieces; with a null
// base it only adds up the size.
struct Carve {
    char *base;
    size_t off = 0;
    template <typename T>
    T *take(size_t count)
    {
        T *p = (T *)(base ? base + off : nullptr);
        off += (count * sizeof(T) + 255) & ~(size_t)255;
        return p;
    }
};

}  // namespace mg
