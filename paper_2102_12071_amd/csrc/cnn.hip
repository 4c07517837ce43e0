// Smoother inference (paper section 4.2: a convolutional network maps the
// field of operator stencils to per-point smoothing kernels).  Network input
// x0 = A / a_C (nine channels), 3x3 "same" convolutions with zero padding at
// every layer, ReLU between layers; output W = omega*delta_0 + y (a damped
// Jacobi term plus the network's correction, so that a zero last layer is
// exactly damped Jacobi, the initialisation the paper uses in section 6.1);
// stored as H = W / a_C.
//
// This file holds the direct (VALU) path used in FP64 precision and the
// smoother field conversions.  The BF16 MFMA path is in cnn_mfma.hip.
#include "common.hpp"
#include "launch.hpp"

namespace mg {

namespace {

template <typename T>
__global__ void k_cnn_input(int n, int P, int64_t plane, const T *A, T *x0)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= n || j >= n) return;
    const int64_t p = (int64_t)j * P + i;
    const T ac = A[kCentre * plane + p];
#pragma unroll
    for (int c = 0; c < 9; ++c) x0[c * plane + p] = A[c * plane + p] / ac;
}

// out[co] = b[co] + sum_ci sum_{ky,kx} w[co][ci][ky][kx] in[ci](j+ky-1, i+kx-1).
// One thread per (node, output channel); weights are read through the cache.
template <typename T>
__global__ void k_conv3x3_direct(int n, int P, int64_t plane, int cin, const T *w, const T *b, const T *in, T *out,
                                 int relu)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int co = blockIdx.z;
    if (i >= n || j >= n) return;
    T acc = b[co];
    for (int ci = 0; ci < cin; ++ci) {
        const T *x = in + ci * plane;
        const T *wk = w + ((int64_t)co * cin + ci) * 9;
#pragma unroll
        for (int ky = 0; ky < 3; ++ky) {
            const int jj = j + ky - 1;
            if (jj < 0 || jj >= n) continue;
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
                const int ii = i + kx - 1;
                if (ii < 0 || ii >= n) continue;
                acc += wk[ky * 3 + kx] * x[(int64_t)jj * P + ii];
            }
        }
    }
    if (relu && !(acc > (T)0)) acc = 0;
    out[co * plane + (int64_t)j * P + i] = acc;
}

template <typename T>
__global__ void k_cnn_output(int n, int P, int64_t plane, const T *A, const T *y, T omega,
                             typename SmootherStore<T>::type *H)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= n || j >= n) return;
    const int64_t p = (int64_t)j * P + i;
    const T ac = A[kCentre * plane + p];
    // a diffusion row's off-centre entries sum to a negative value; other rows (Dirichlet nodes of a
    // masked domain and their Galerkin images) take damped Jacobi.  Summed in channel order.
    T off = 0;
#pragma unroll
    for (int c = 0; c < kStencil; ++c)
        if (c != kCentre) off += A[c * plane + p];
    const bool diffusion = off < (T)0;
#pragma unroll
    for (int k = 0; k < kSmoother; ++k) {
        const T wv = (diffusion ? y[k * plane + p] : (T)0) + (k == 12 ? omega : (T)0);
        store_h(H + k * plane + p, wv / ac);
    }
}

template <typename T>
__global__ void k_set_smoother(int n, int P, int64_t plane, const double *W, int Pw, int64_t planew,
                               const double *A64, typename SmootherStore<T>::type *H)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= n || j >= n) return;
    const int64_t p = (int64_t)j * P + i;
    const double ac = A64[kCentre * plane + p];
    for (int k = 0; k < kSmoother; ++k) store_h(H + k * plane + p, (T)(W[k * planew + (int64_t)j * Pw + i] / ac));
}

// Damped Jacobi as a 5x5 smoother field: W = omega * delta_0, so H = W / a_C
// holds omega / a_C at the centre tap and zero elsewhere (the fallback of a
// problem whose learned smoother stalls or diverges).
template <typename T>
__global__ void k_jacobi_smoother(int n, int P, int64_t plane, const double *A64, double omega,
                                  typename SmootherStore<T>::type *H)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= n || j >= n) return;
    const int64_t p = (int64_t)j * P + i;
    const double ac = A64[kCentre * plane + p];
    for (int k = 0; k < kSmoother; ++k) store_h(H + k * plane + p, (T)(k == kSmoother / 2 ? omega / ac : 0.0));
}

template <typename T>
__global__ void k_get_smoother(int n, int P, int64_t plane, const typename SmootherStore<T>::type *H,
                               const double *A64, double *W, int Pw, int64_t planew)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= n || j >= n) return;
    const int64_t p = (int64_t)j * P + i;
    const double ac = A64[kCentre * plane + p];
    for (int k = 0; k < kSmoother; ++k) W[k * planew + (int64_t)j * Pw + i] = (double)load_h(H + k * plane + p) * ac;
}

__global__ void k_f32_to_f64(int64_t count, const float *src, double *dst)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < count) dst[q] = (double)src[q];
}

inline dim3 grid2(int n, dim3 blk, int z = 1) { return dim3((n + blk.x - 1) / blk.x, (n + blk.y - 1) / blk.y, z); }

}  // namespace

template <typename T>
void launch_cnn_input(int n, int P, int64_t plane, const T *A, T *x0, hipStream_t st)
{
    dim3 blk(64, 4);
    k_cnn_input<T><<<grid2(n, blk), blk, 0, st>>>(n, P, plane, A, x0);
}

template <typename T>
void launch_conv3x3_direct(int n, int P, int64_t plane, int cin, int cout, const T *w, const T *b, const T *in,
                           T *out, bool relu, hipStream_t st)
{
    dim3 blk(64, 4);
    k_conv3x3_direct<T><<<grid2(n, blk, cout), blk, 0, st>>>(n, P, plane, cin, w, b, in, out, relu ? 1 : 0);
}

template <typename T>
void launch_cnn_output(int n, int P, int64_t plane, const T *A, const T *y, double omega,
                       typename SmootherStore<T>::type *H, hipStream_t st)
{
    dim3 blk(64, 4);
    k_cnn_output<T><<<grid2(n, blk), blk, 0, st>>>(n, P, plane, A, y, (T)omega, H);
}

template <typename T>
void launch_set_smoother(int n, int P, int64_t plane, const double *W, int Pw, int64_t planew, const double *A64,
                         typename SmootherStore<T>::type *H, hipStream_t st)
{
    dim3 blk(64, 4);
    k_set_smoother<T><<<grid2(n, blk), blk, 0, st>>>(n, P, plane, W, Pw, planew, A64, H);
}

template <typename T>
void launch_jacobi_smoother(int n, int P, int64_t plane, const double *A64, double omega,
                            typename SmootherStore<T>::type *H, hipStream_t st)
{
    dim3 blk(64, 4);
    k_jacobi_smoother<T><<<grid2(n, blk), blk, 0, st>>>(n, P, plane, A64, omega, H);
}

template <typename T>
void launch_get_smoother(int n, int P, int64_t plane, const typename SmootherStore<T>::type *H,
                         const double *A64, double *W, int Pw, int64_t planew, hipStream_t st)
{
    dim3 blk(64, 4);
    k_get_smoother<T><<<grid2(n, blk), blk, 0, st>>>(n, P, plane, H, A64, W, Pw, planew);
}

void launch_f32_to_f64(int64_t count, const float *src, double *dst, hipStream_t st)
{
    k_f32_to_f64<<<(unsigned)((count + 255) / 256), 256, 0, st>>>(count, src, dst);
}

#define MG_INSTANTIATE(T)                                                                                         \
    template void launch_cnn_input<T>(int, int, int64_t, const T *, T *, hipStream_t);                            \
    template void launch_conv3x3_direct<T>(int, int, int64_t, int, int, const T *, const T *, const T *, T *,      \
                                           bool, hipStream_t);                                                    \
    template void launch_cnn_output<T>(int, int, int64_t, const T *, const T *, double,                           \
                                       typename SmootherStore<T>::type *, hipStream_t);                           \
    template void launch_set_smoother<T>(int, int, int64_t, const double *, int, int64_t, const double *,         \
                                         typename SmootherStore<T>::type *, hipStream_t);                         \
    template void launch_get_smoother<T>(int, int, int64_t, const typename SmootherStore<T>::type *,              \
                                         const double *, double *, int, int64_t, hipStream_t);                     \
    template void launch_jacobi_smoother<T>(int, int, int64_t, const double *, double,                            \
                                            typename SmootherStore<T>::type *, hipStream_t);
MG_INSTANTIATE(float)
MG_INSTANTIATE(double)
#undef MG_INSTANTIATE

}  // namespace mg
