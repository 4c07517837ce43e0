// Kernels of the adaptive training step (Algorithm 2): the forward cycles on
// the trained level and their adjoint, batched over the problems of a
// training stage, all of one size n (blockIdx.z = problem).  FP64.
//
// Level vectors of the step's workspace: rows of pitch P = n + 1, problem z
// at offset z * vs.  The trained level's stencil A and smoother H = W / a_C
// come from the top context's finest level; the coarse right-hand side and
// correction live in a coarse context's finest-level buffers (pitch Pc =
// nc + 1).  Every node (i, j) with i, j < n is written; padding is not read.
#include "alpha.hpp"

namespace mg {

namespace {

constexpr int kAT = 256;

__device__ inline bool inside(int n, int i, int j) { return i >= 0 && i < n && j >= 0 && j < n; }

// The node of this thread: flat index over the n x n interior of problem blockIdx.z.
struct Node {
    int i, j, z;
    bool ok;
};
__device__ inline Node node_of(int n)
{
    const int q = blockIdx.x * kAT + threadIdx.x;
    return Node{q % n, q / n, (int)blockIdx.z, q < n * n};
}

// y = b + sign * A x (b null: 0)
__global__ void __launch_bounds__(kAT) k_al_apply_A(const AlphaProb *pr, int n, int P, int64_t plane, int64_t vs,
                                                     const double *x, const double *b, double sign, double *y,
                                                     const int *active)
{
    const Node t = node_of(n);
    if (!t.ok || !active[t.z]) return;
    const int64_t p = (int64_t)t.j * P + t.i, o = t.z * vs;
    const double MG_G *A = pr[t.z].A;
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < 9; ++c) {
        const int ii = t.i + c % 3 - 1, jj = t.j + c / 3 - 1;
        const bool in = inside(n, ii, jj);
        const double xv = x[o + (in ? (int64_t)jj * P + ii : p)];
        acc += A[c * plane + p] * (in ? xv : 0.0);
    }
    y[o + p] = (b ? b[o + p] : 0.0) + sign * acc;
}

// y = (accumulate ? y : 0) + H x, or + H^T x with (H^T x)_p = sum_k H_{p - off(k)}[k] x_{p - off(k)}
template <bool TRANSPOSE>
__global__ void __launch_bounds__(kAT) k_al_H(const AlphaProb *pr, int n, int P, int64_t plane, int64_t vs,
                                               const double *x, double *y, int accumulate, const int *active)
{
    const Node t = node_of(n);
    if (!t.ok || !active[t.z]) return;
    const int64_t p = (int64_t)t.j * P + t.i, o = t.z * vs;
    const double MG_G *H = pr[t.z].H;
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < 25; ++k) {
        const int dx = k % 5 - 2, dy = k / 5 - 2;
        const int ii = TRANSPOSE ? t.i - dx : t.i + dx, jj = TRANSPOSE ? t.j - dy : t.j + dy;
        const bool in = inside(n, ii, jj);
        const int64_t q = in ? (int64_t)jj * P + ii : p;
        const double h = H[k * plane + (TRANSPOSE ? q : p)];
        acc += in ? h * x[o + q] : 0.0;
    }
    y[o + p] = (accumulate ? y[o + p] : 0.0) + acc;
}

// dH_p[k] += g_p x_{p + off(k)}: the gradient of <g, H x> with respect to the field H
__global__ void __launch_bounds__(kAT) k_al_outer(int n, int P, int64_t plane, int64_t vs, const double *g,
                                                   const double *x, double *dH, const int *active)
{
    const Node t = node_of(n);
    if (!t.ok || !active[t.z]) return;
    const int64_t p = (int64_t)t.j * P + t.i, o = t.z * vs, oh = t.z * 25 * plane;
    const double gp = g[o + p];
#pragma unroll
    for (int k = 0; k < 25; ++k) {
        const int ii = t.i + k % 5 - 2, jj = t.j + k / 5 - 2;
        const bool in = inside(n, ii, jj);
        const double xv = x[o + (in ? (int64_t)jj * P + ii : p)];
        dH[oh + k * plane + p] += in ? gp * xv : 0.0;
    }
}

// rc = R x (full weighting) into the coarse context's right-hand side, and
// its solution cleared: the coarse cycle then returns Psi_c(R x).
__global__ void __launch_bounds__(kAT) k_al_restrict(const AlphaProb *pr, int which, int n, int P, int64_t vs,
                                                      const double *x, const int *active)
{
    const int nc = (n - 1) / 2, Pc = nc + 1;
    const Node t = node_of(nc);
    if (!t.ok || !active[t.z]) return;
    const double *v = x + t.z * vs;
    const int64_t c = (int64_t)(2 * t.j + 1) * P + 2 * t.i + 1;  // interior: c +- P +- 1 stay on the grid
    const double r = 0.0625 * (v[c - P - 1] + v[c - P + 1] + v[c + P - 1] + v[c + P + 1]) +
                     0.125 * (v[c - P] + v[c + P] + v[c - 1] + v[c + 1]) + 0.25 * v[c];
    const int64_t pc = (int64_t)t.j * Pc + t.i;
    pr[t.z].rc[which][pc] = r;
    pr[t.z].uc[which][pc] = 0.0;
}

// y = (x ? x : 0) + P ec, bilinear, ec the coarse context's solution
__global__ void __launch_bounds__(kAT) k_al_prolong(const AlphaProb *pr, int which, int n, int P, int64_t vs,
                                                     const double *x, double *y, const int *active)
{
    const Node t = node_of(n);
    if (!t.ok || !active[t.z]) return;
    const int nc = (n - 1) / 2, Pc = nc + 1;
    const double MG_G *e = pr[t.z].uc[which];
    // coarse node I sits on fine node 2I+1: odd coordinates have one coarse
    // neighbour (weight 1), even ones the two around them (weight 1/2 each)
    const int i = t.i, j = t.j;
    const int ia = (i & 1) ? (i - 1) / 2 : i / 2 - 1, ib = (i & 1) ? ia : ia + 1;
    const int ja = (j & 1) ? (j - 1) / 2 : j / 2 - 1, jb = (j & 1) ? ja : ja + 1;
    auto at = [&](int I, int J) {
        return (I >= 0 && I < nc && J >= 0 && J < nc) ? e[(int64_t)J * Pc + I] : 0.0;
    };
    double acc = at(ia, ja);
    if (ib != ia) acc += at(ib, ja);
    if (jb != ja) {
        acc += at(ia, jb);
        if (ib != ia) acc += at(ib, jb);
    }
    const double wt = ((i & 1) ? 1.0 : 0.5) * ((j & 1) ? 1.0 : 0.5);
    const int64_t p = t.z * vs + (int64_t)j * P + i;
    y[p] = (x ? x[p] : 0.0) + wt * acc;
}

// y = x + s w
__global__ void __launch_bounds__(kAT) k_al_axpy(int n, int P, int64_t vs, const double *x, double s, const double *w,
                                                  double *y, const int *active)
{
    const Node t = node_of(n);
    if (!t.ok || !active[t.z]) return;
    const int64_t p = t.z * vs + (int64_t)t.j * P + t.i;
    y[p] = x[p] + s * w[p];
}

// dist[z] = ||x - y||_2 over the interior (one block per problem, fixed order)
__global__ void __launch_bounds__(kAT) k_al_dist(int n, int P, int64_t vs, const double *x, const double *y,
                                                  double *dist)
{
    __shared__ double red[kAT / 64];
    const int z = blockIdx.x;
    double acc = 0.0;
    for (int q = threadIdx.x; q < n * n; q += kAT) {
        const int64_t p = z * vs + (int64_t)(q / n) * P + q % n;
        const double d = x[p] - y[p];
        acc += d * d;
    }
    const double s = block_sum<kAT>(acc, red);
    if (threadIdx.x == 0) dist[z] = sqrt(s);
}

// lam = scale (x - y) / dist[z], zero where dist[z] = 0; dH = 0 (when given)
__global__ void __launch_bounds__(kAT) k_al_seed(int n, int P, int64_t plane, int64_t vs, const double *x,
                                                  const double *y, const double *dist, double scale, double *lam,
                                                  double *dH)
{
    const Node t = node_of(n);
    if (!t.ok) return;
    const int64_t p = t.z * vs + (int64_t)t.j * P + t.i;
    const double d = dist[t.z];
    lam[p] = d > 0.0 ? scale * (x[p] - y[p]) / d : 0.0;
    if (!dH) return;
    const int64_t oh = t.z * 25 * plane + (int64_t)t.j * P + t.i;
    for (int k = 0; k < 25; ++k) dH[oh + k * plane] = 0.0;
}

// dW = dH / a_C (W = a_C H): FP32 into out ([25][n*n] per problem, stride
// 25 n^2), the network's output gradient, and FP64 into W64[z] ([25][n][n])
// when W64 is given
__global__ void __launch_bounds__(kAT) k_al_dw(const AlphaProb *pr, int n, int P, int64_t plane, const double *dH,
                                                double *const *W64, float *out)
{
    const Node t = node_of(n);
    if (!t.ok) return;
    const int64_t p = (int64_t)t.j * P + t.i, oh = t.z * 25 * plane, d = (int64_t)t.j * n + t.i;
    const int64_t nn = (int64_t)n * n;
    const double ac = pr[t.z].A[kCentre * plane + p];
    double *w64 = W64 ? W64[t.z] : nullptr;
    float *o = out + t.z * 25 * nn;
    for (int k = 0; k < 25; ++k) {
        const double g = dH[oh + k * plane + p] / ac;
        o[k * nn + d] = (float)g;
        if (w64) w64[k * nn + d] = g;
    }
}

// WT_p[k] = a_C(p) W_{p + off(k)}[24 - k] / a_C(p + off(k)) (zero off the
// grid): the field whose smoother is H^T.  Dense [25][n][n] in and out.
__global__ void __launch_bounds__(kAT) k_al_transpose(int n, const double *A, const double *W, double *WT)
{
    const int q = blockIdx.x * kAT + threadIdx.x;
    if (q >= n * n) return;
    const int i = q % n, j = q / n;
    const int64_t nn = (int64_t)n * n;
    const double ac = A[kCentre * nn + q];
    for (int k = 0; k < 25; ++k) {
        const int ii = i + k % 5 - 2, jj = j + k / 5 - 2;
        double v = 0.0;
        if (inside(n, ii, jj)) {
            const int64_t s = (int64_t)jj * n + ii;
            v = ac * W[(24 - k) * nn + s] / A[kCentre * nn + s];
        }
        WT[k * nn + q] = v;
    }
}

inline dim3 grid_of(int n, int nb) { return dim3((unsigned)(((int64_t)n * n + kAT - 1) / kAT), 1, nb); }

}  // namespace

void launch_al_apply_A(const AlphaProb *pr, int nb, int n, int P, int64_t plane, int64_t vs, const double *x,
                       const double *b, double sign, double *y, const int *active, hipStream_t st)
{
    k_al_apply_A<<<grid_of(n, nb), kAT, 0, st>>>(pr, n, P, plane, vs, x, b, sign, y, active);
}

void launch_al_H(const AlphaProb *pr, int nb, int n, int P, int64_t plane, int64_t vs, const double *x, double *y,
                 bool transpose, bool accumulate, const int *active, hipStream_t st)
{
    if (transpose)
        k_al_H<true><<<grid_of(n, nb), kAT, 0, st>>>(pr, n, P, plane, vs, x, y, accumulate, active);
    else
        k_al_H<false><<<grid_of(n, nb), kAT, 0, st>>>(pr, n, P, plane, vs, x, y, accumulate, active);
}

void launch_al_outer(int nb, int n, int P, int64_t plane, int64_t vs, const double *g, const double *x, double *dH,
                     const int *active, hipStream_t st)
{
    k_al_outer<<<grid_of(n, nb), kAT, 0, st>>>(n, P, plane, vs, g, x, dH, active);
}

void launch_al_restrict(const AlphaProb *pr, int which, int nb, int n, int P, int64_t vs, const double *x,
                        const int *active, hipStream_t st)
{
    k_al_restrict<<<grid_of((n - 1) / 2, nb), kAT, 0, st>>>(pr, which, n, P, vs, x, active);
}

void launch_al_prolong(const AlphaProb *pr, int which, int nb, int n, int P, int64_t vs, const double *x, double *y,
                       const int *active, hipStream_t st)
{
    k_al_prolong<<<grid_of(n, nb), kAT, 0, st>>>(pr, which, n, P, vs, x, y, active);
}

void launch_al_axpy(int nb, int n, int P, int64_t vs, const double *x, double s, const double *w, double *y,
                    const int *active, hipStream_t st)
{
    k_al_axpy<<<grid_of(n, nb), kAT, 0, st>>>(n, P, vs, x, s, w, y, active);
}

void launch_al_dist(int nb, int n, int P, int64_t vs, const double *x, const double *y, double *dist, hipStream_t st)
{
    k_al_dist<<<nb, kAT, 0, st>>>(n, P, vs, x, y, dist);
}

void launch_al_seed(int nb, int n, int P, int64_t plane, int64_t vs, const double *x, const double *y,
                    const double *dist, double scale, double *lam, double *dH, hipStream_t st)
{
    k_al_seed<<<grid_of(n, nb), kAT, 0, st>>>(n, P, plane, vs, x, y, dist, scale, lam, dH);
}

void launch_al_dw(const AlphaProb *pr, int nb, int n, int P, int64_t plane, const double *dH, double *const *W64,
                  float *out, hipStream_t st)
{
    k_al_dw<<<grid_of(n, nb), kAT, 0, st>>>(pr, n, P, plane, dH, W64, out);
}

void launch_al_transpose(int n, const double *A, const double *W, double *WT, hipStream_t st)
{
    k_al_transpose<<<grid_of(n, 1), kAT, 0, st>>>(n, A, W, WT);
}

}  // namespace mg
