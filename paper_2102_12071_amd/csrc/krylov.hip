// Vector kernels of the flexible-GMRES outer solver (section 6, multigrid
// cycles as the preconditioner of flexible GMRES).  Every vector is FP64 on
// the finest grid of one problem: rows of pitch P = n + 1 (a power of two),
// n*P elements, the padding column zero.  Kernels only touch interior nodes,
// so the padding stays zero.  Reductions are deterministic: fixed-size
// partial sums per block, then one block sums them in a fixed order.
#include <mutex>

#include "common.hpp"
#include "launch.hpp"

namespace mg {

// The fixed workspace of mg_solve_fgmres_noalloc (callers that cannot allocate
// device memory): one array per GPU, loaded with this code object and held
// until the process ends.  Host code never passes the array's name to a
// kernel: it takes the device address hipGetSymbolAddress gives, once per
// device, with that device current.
static __device__ __align__(256) double scratch[kKrylovStaticBytes / sizeof(double)];

namespace {
constexpr int kMaxStaticDevices = 64;
std::mutex g_scratch_mutex;
double *g_scratch_ptr[kMaxStaticDevices] = {};
}  // namespace

hipError_t krylov_static_workspace(double **ptr)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxStaticDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

namespace {

constexpr int kKT = 256;

// y = b + sign * (A x) on the interior (b may be null: y = sign * A x)
__global__ void __launch_bounds__(kKT) k_kr_apply(int n, int P, int64_t plane, const double *A, const double *x,
                                                   const double *b, double sign, double *y)
{
    const int i = blockIdx.x * kKT + threadIdx.x, j = blockIdx.y;
    if (i >= n) return;
    const int64_t p = (int64_t)j * P + i;
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < 9; ++c) {
        const int ii = i + c % 3 - 1, jj = j + c / 3 - 1;
        const bool ok = ii >= 0 && ii < n && jj >= 0 && jj < n;
        const double xv = x[ok ? (int64_t)jj * P + ii : p];  // unconditional load, then select
        acc += A[c * plane + p] * (ok ? xv : 0.0);
    }
    y[p] = (b ? b[p] : 0.0) + sign * acc;
}

// partial[v * nb + blk] = sum over this block's share of <w, V_v> (V_v = V + v * vstride)
__global__ void __launch_bounds__(kKT) k_kr_dots(int64_t len, int P, int n, const double *w, const double *V,
                                                  int64_t vstride, double *partial)
{
    __shared__ double red[kKT / 64];
    const int v = blockIdx.y, nb = gridDim.x;
    const double *x = V + v * vstride;
    double acc = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * kKT + threadIdx.x; p < len; p += (int64_t)nb * kKT)
        if ((int)(p & (P - 1)) < n) acc += w[p] * x[p];
    const double s = block_sum<kKT>(acc, red);
    if (threadIdx.x == 0) partial[(int64_t)v * nb + blockIdx.x] = s;
}

// out[v] = sum_b partial[v * nb + b], in order; scale: out[v] = sqrt(sum) when root
__global__ void __launch_bounds__(kKT) k_kr_reduce(const double *partial, int nb, double *out, int root)
{
    __shared__ double red[kKT / 64];
    const int v = blockIdx.x;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += kKT) acc += partial[(int64_t)v * nb + b];
    const double s = block_sum<kKT>(acc, red);
    if (threadIdx.x == 0) out[v] = root ? sqrt(s) : s;
}

// w -= sum_v coef[v] V_v
__global__ void __launch_bounds__(kKT) k_kr_update(int n, int P, double *w, const double *V, int64_t vstride, int nv,
                                                    const double *coef)
{
    const int i = blockIdx.x * kKT + threadIdx.x, j = blockIdx.y;
    if (i >= n) return;
    const int64_t p = (int64_t)j * P + i;
    double acc = w[p];
    for (int v = 0; v < nv; ++v) acc -= coef[v] * V[v * vstride + p];
    w[p] = acc;
}

// y = x / (*d)
__global__ void __launch_bounds__(kKT) k_kr_scale(int n, int P, const double *x, const double *d, double *y)
{
    const int i = blockIdx.x * kKT + threadIdx.x, j = blockIdx.y;
    if (i >= n) return;
    const int64_t p = (int64_t)j * P + i;
    y[p] = x[p] / *d;
}

// u += sum_k coef[k] Z_k
__global__ void __launch_bounds__(kKT) k_kr_combine(int n, int P, double *u, const double *Z, int64_t vstride, int nz,
                                                     const double *coef)
{
    const int i = blockIdx.x * kKT + threadIdx.x, j = blockIdx.y;
    if (i >= n) return;
    const int64_t p = (int64_t)j * P + i;
    double acc = u[p];
    for (int k = 0; k < nz; ++k) acc += coef[k] * Z[k * vstride + p];
    u[p] = acc;
}

inline dim3 rows_grid(int n) { return dim3((n + kKT - 1) / kKT, n); }

}  // namespace

void launch_kr_apply(int n, int P, int64_t plane, const double *A, const double *x, const double *b, double sign,
                     double *y, hipStream_t st)
{
    k_kr_apply<<<rows_grid(n), kKT, 0, st>>>(n, P, plane, A, x, b, sign, y);
}

void launch_kr_dots(int n, int P, const double *w, const double *V, int64_t vstride, int nv, double *partial,
                    double *out, int root, hipStream_t st)
{
    const int64_t len = (int64_t)n * P;
    const int nb = kKrylovBlocks;
    k_kr_dots<<<dim3(nb, nv), kKT, 0, st>>>(len, P, n, w, V, vstride, partial);
    k_kr_reduce<<<nv, kKT, 0, st>>>(partial, nb, out, root);
}

void launch_kr_update(int n, int P, double *w, const double *V, int64_t vstride, int nv, const double *coef,
                      hipStream_t st)
{
    k_kr_update<<<rows_grid(n), kKT, 0, st>>>(n, P, w, V, vstride, nv, coef);
}

void launch_kr_scale(int n, int P, const double *x, const double *d, double *y, hipStream_t st)
{
    k_kr_scale<<<rows_grid(n), kKT, 0, st>>>(n, P, x, d, y);
}

void launch_kr_combine(int n, int P, double *u, const double *Z, int64_t vstride, int nz, const double *coef,
                       hipStream_t st)
{
    k_kr_combine<<<rows_grid(n), kKT, 0, st>>>(n, P, u, Z, vstride, nz, coef);
}

}  // namespace mg
