// Discretisation and coarsening kernels (setup path):
//  * bilinear (Q1) nine-point stencil of the rotated anisotropic operator
//    (paper section 4 stencil; section 6 tensor T(theta, xi));
//  * five-point stencil of -div(a grad u) with face-averaged cell coefficients;
//  * Galerkin coarse stencils Ac = R A P (section 2.2) in stencil form;
//  * layout copies, FP64 -> FP32 conversion and input validation.
// All in FP64; one thread per output node.  These run once per problem.
#include "common.hpp"
#include "launch.hpp"

namespace mg {

namespace {

__device__ inline bool inside(int n, int i, int j) { return i >= 0 && i < n && j >= 0 && j < n; }

__global__ void k_q1_rotated(int n, int P, int64_t plane, double k11, double k12, double k22, double *out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= n || j >= n) return;
    // Element integrals of the bilinear basis: each of the four cells around
    // the node adds (k11+k22)/3 +- k12/2 to the centre, -k11/3 + k22/6 to the
    // x-neighbour on its side, k11/6 - k22/3 to the y-neighbour on its side
    // and -(k11+k22)/6 -+ k12/2 to the diagonal neighbour it contains.
    const double edge_x = -k11 / 3.0 + k22 / 6.0;
    const double edge_y = k11 / 6.0 - k22 / 3.0;
    double v[9];
    v[4] = 4.0 * (k11 + k22) / 3.0;
    v[3] = v[5] = 2.0 * edge_x;
    v[1] = v[7] = 2.0 * edge_y;
    v[0] = v[8] = -(k11 + k22) / 6.0 - 0.5 * k12;  // SW, NE: cells where sx*sy = +1
    v[2] = v[6] = -(k11 + k22) / 6.0 + 0.5 * k12;  // SE, NW
#pragma unroll
    for (int c = 0; c < 9; ++c) {
        const int dx = c % 3 - 1, dy = c / 3 - 1;
        out[c * plane + (int64_t)j * P + i] = inside(n, i + dx, j + dy) ? v[c] : 0.0;
    }
}

// The same stencil for a batch of problems of one size, the tensor of problem z
// at k[3 z .. 3 z + 2] (k11, k12, k22); out: [count][9][n][n].
__global__ void k_q1_rotated_batch(int n, const double *k, double *out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= n || j >= n) return;
    const double k11 = k[3 * blockIdx.z], k12 = k[3 * blockIdx.z + 1], k22 = k[3 * blockIdx.z + 2];
    const int64_t plane = (int64_t)n * n;
    double *o = out + (int64_t)blockIdx.z * 9 * plane;
    const double edge_x = -k11 / 3.0 + k22 / 6.0;
    const double edge_y = k11 / 6.0 - k22 / 3.0;
    double v[9];
    v[4] = 4.0 * (k11 + k22) / 3.0;
    v[3] = v[5] = 2.0 * edge_x;
    v[1] = v[7] = 2.0 * edge_y;
    v[0] = v[8] = -(k11 + k22) / 6.0 - 0.5 * k12;
    v[2] = v[6] = -(k11 + k22) / 6.0 + 0.5 * k12;
#pragma unroll
    for (int c = 0; c < 9; ++c) {
        const int dx = c % 3 - 1, dy = c / 3 - 1;
        o[c * plane + (int64_t)j * n + i] = inside(n, i + dx, j + dy) ? v[c] : 0.0;
    }
}

__global__ void k_cellavg5(int n, const double *a, int Pa, int P, int64_t plane, double *out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= n || j >= n) return;
    // cells around node (i, j): SW (i, j), SE (i+1, j), NW (i, j+1), NE (i+1, j+1)
    const double sw = a[(int64_t)j * Pa + i], se = a[(int64_t)j * Pa + i + 1];
    const double nw = a[(int64_t)(j + 1) * Pa + i], ne = a[(int64_t)(j + 1) * Pa + i + 1];
    const double aE = 0.5 * (se + ne), aW = 0.5 * (sw + nw), aN = 0.5 * (nw + ne), aS = 0.5 * (sw + se);
    const int64_t p = (int64_t)j * P + i;
    out[0 * plane + p] = 0.0;
    out[2 * plane + p] = 0.0;
    out[6 * plane + p] = 0.0;
    out[8 * plane + p] = 0.0;
    out[4 * plane + p] = aE + aW + aN + aS;
    out[5 * plane + p] = (i + 1 < n) ? -aE : 0.0;
    out[3 * plane + p] = (i > 0) ? -aW : 0.0;
    out[7 * plane + p] = (j + 1 < n) ? -aN : 0.0;
    out[1 * plane + p] = (j > 0) ? -aS : 0.0;
}

// Bilinear weight of a fine node at offset (bx, by) from a coarse node.
__device__ inline double bilinear_w(int bx, int by)
{
    if (bx < -1 || bx > 1 || by < -1 || by > 1) return 0.0;
    return (bx == 0 ? 1.0 : 0.5) * (by == 0 ? 1.0 : 0.5);
}

// Ac_I[D] = sum_{a in [-1,1]^2} (w(a)/4) sum_{d in [-1,1]^2} A_{2I+1+a}[d] w(a + d - 2D),
// zero when the coarse neighbour I + D is outside the coarse grid.  The fine nodes a are taken one at
// a time (their nine entries, the nine sums acc[D] carried along): each acc[D] adds its terms in the
// order of a and each inner sum in the order of d, as the definition is written (the same values as
// the form that held all 81 entries, bit for bit).  The launch bound matches the 128-thread blocks:
// without it the compiler kept to 128 registers and spilled (restencil at n = 4095: 3.9 -> 2.2 ms).
__global__ void __launch_bounds__(128) k_galerkin(int n, int P, int64_t plane, const double *A, int nc, int Pc,
                                                  int64_t planec, double *Ac)
{
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int J = blockIdx.y * blockDim.y + threadIdx.y;
    if (I >= nc || J >= nc) return;
    double acc[9];
#pragma unroll
    for (int D = 0; D < 9; ++D) acc[D] = 0.0;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int ax = t % 3 - 1, ay = t / 3 - 1;
        const int xi = 2 * I + 1 + ax, xj = 2 * J + 1 + ay;
        double a[9];  // the fine stencil of fine node t around the coarse node
#pragma unroll
        for (int c = 0; c < 9; ++c) a[c] = A[c * plane + (int64_t)xj * P + xi];
        const double wr = 0.25 * bilinear_w(ax, ay);
#pragma unroll
        for (int D = 0; D < 9; ++D) {
            const int Dx = D % 3 - 1, Dy = D / 3 - 1;
            double inner = 0.0;
#pragma unroll
            for (int c = 0; c < 9; ++c) {
                const int dx = c % 3 - 1, dy = c / 3 - 1;
                inner += a[c] * bilinear_w(ax + dx - 2 * Dx, ay + dy - 2 * Dy);
            }
            acc[D] += wr * inner;
        }
    }
#pragma unroll
    for (int D = 0; D < 9; ++D) {
        const int Dx = D % 3 - 1, Dy = D / 3 - 1;
        Ac[D * planec + (int64_t)J * Pc + I] = inside(nc, I + Dx, J + Dy) ? acc[D] : 0.0;
    }
}

__global__ void k_copy_field(int n, int nch, const double *src, int Ps, int64_t planes, double *dst, int Pd,
                             int64_t planed)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= n || j >= n) return;
    for (int c = 0; c < nch; ++c) dst[c * planed + (int64_t)j * Pd + i] = src[c * planes + (int64_t)j * Ps + i];
}

__global__ void k_to_f32(int64_t count, const double *src, float *dst)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < count) dst[q] = (float)src[q];
}

// flag bit 1: an entry couples to a node outside the grid; bit 2: centre <= 0
// or not finite; bit 4: an entry is not finite.
__global__ void k_validate(int n, int P, int64_t plane, const double *A, int *flag)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= n || j >= n) return;
    int bad = 0;
    for (int c = 0; c < 9; ++c) {
        const double v = A[c * plane + (int64_t)j * P + i];
        if (!isfinite(v)) bad |= 4;
        if (!inside(n, i + c % 3 - 1, j + c / 3 - 1) && v != 0.0) bad |= 1;
    }
    const double ac = A[kCentre * plane + (int64_t)j * P + i];
    if (!(ac > 0.0)) bad |= 2;
    if (bad) atomicOr(flag, bad);
}

// Level 0 of a problem from the caller's dense [9][n][n] stencil in one pass
// over it: the pitched FP64 copy, its FP32 copy (A32 not null), the checks of
// k_validate, and the symmetry flags, A[c](p) == A[8-c](p + d_c) wherever both
// nodes are on the grid, of the FP64 entries (sym64) and of the ones the cycle
// reads (symc: their FP32 roundings when A32 is given, else the FP64 ones).
// Both flags start at 1 (k_flags_init); a node that fails writes 0.
__global__ void k_flags_init(int *a, int *b)
{
    *a = 1;
    *b = 1;
}
__global__ void k_ingest(int n, const double *src, int P, int64_t plane, double *A64, float *A32, int *flag,
                         int *sym64, int *symc)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= n || j >= n) return;
    const int64_t nn = (int64_t)n * n, q = (int64_t)j * n + i, p = (int64_t)j * P + i;
    double v[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) v[c] = src[c * nn + q];
    int bad = 0;
#pragma unroll
    for (int c = 0; c < 9; ++c) {
        if (!isfinite(v[c])) bad |= 4;
        if (!inside(n, i + c % 3 - 1, j + c / 3 - 1) && v[c] != 0.0) bad |= 1;
        A64[c * plane + p] = v[c];
        if (A32) A32[c * plane + p] = (float)v[c];
    }
    if (!(v[kCentre] > 0.0)) bad |= 2;
    if (bad) atomicOr(flag, bad);
    bool s64 = true, s32 = true;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int ii = i + c % 3 - 1, jj = j + c / 3 - 1;
        if (!inside(n, ii, jj)) continue;
        const double m = src[(8 - c) * nn + (int64_t)jj * n + ii];
        s64 = s64 && v[c] == m;
        s32 = s32 && (float)v[c] == (float)m;
    }
    if (!s64) *sym64 = 0;  // every writer writes 0
    if (!(A32 ? s32 : s64)) *symc = 0;
}

// Dirichlet condition on the nodes outside a domain (mask 0): their rows keep
// only the centre entry, and the rows of the nodes inside drop the couplings to
// them.  Dense [9][n][n] in and out (may alias: each thread reads and writes
// its own node only).
__global__ void k_mask(int n, const uint8_t *mask, const double *A, double *out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= n || j >= n) return;
    const int64_t nn = (int64_t)n * n, p = (int64_t)j * n + i;
    const bool in = mask[p] != 0;
    for (int c = 0; c < 9; ++c) {
        const int ii = i + c % 3 - 1, jj = j + c / 3 - 1;
        double v = A[c * nn + p];
        if (c != kCentre) {
            const bool nb_in = inside(n, ii, jj) && mask[(int64_t)jj * n + ii] != 0;
            if (!in || !nb_in) v = 0.0;
        }
        out[c * nn + p] = v;
    }
}

dim3 node_grid(int n, dim3 blk) { return dim3((n + blk.x - 1) / blk.x, (n + blk.y - 1) / blk.y, 1); }

}  // namespace

void q1_tensor(double theta, double eps, double *k)
{
    const double c = cos(theta), s = sin(theta);
    k[0] = c * c + eps * s * s;
    k[1] = c * s * (1.0 - eps);
    k[2] = s * s + eps * c * c;
}

void launch_q1_rotated(int n, int P, int64_t plane, double theta, double eps, double *out, hipStream_t st)
{
    double k[3];
    q1_tensor(theta, eps, k);
    dim3 blk(64, 4);
    k_q1_rotated<<<node_grid(n, blk), blk, 0, st>>>(n, P, plane, k[0], k[1], k[2], out);
}

void launch_q1_rotated_batch(int n, int count, const double *k, double *out, hipStream_t st)
{
    dim3 blk(64, 4);
    dim3 g = node_grid(n, blk);
    g.z = count;
    k_q1_rotated_batch<<<g, blk, 0, st>>>(n, k, out);
}

void launch_cellavg5(int n, const double *a, int Pa, int P, int64_t plane, double *out, hipStream_t st)
{
    dim3 blk(64, 4);
    k_cellavg5<<<node_grid(n, blk), blk, 0, st>>>(n, a, Pa, P, plane, out);
}

void launch_galerkin(int n, int P, int64_t plane, const double *A, int Pc, int64_t planec, double *Ac,
                     hipStream_t st)
{
    const int nc = (n - 1) / 2;
    dim3 blk(64, 2);  // 128 threads: the kernel's launch bound
    k_galerkin<<<node_grid(nc, blk), blk, 0, st>>>(n, P, plane, A, nc, Pc, planec, Ac);
}

void launch_copy_field(int n, int nch, const double *src, int Ps, int64_t planes, double *dst, int Pd,
                       int64_t planed, hipStream_t st)
{
    dim3 blk(64, 4);
    k_copy_field<<<node_grid(n, blk), blk, 0, st>>>(n, nch, src, Ps, planes, dst, Pd, planed);
}

void launch_to_f32(int64_t count, const double *src, float *dst, hipStream_t st)
{
    const int nt = 256;
    k_to_f32<<<(unsigned)((count + nt - 1) / nt), nt, 0, st>>>(count, src, dst);
}

void launch_mask(int n, const uint8_t *mask, const double *A, double *out, hipStream_t st)
{
    dim3 blk(64, 4);
    k_mask<<<node_grid(n, blk), blk, 0, st>>>(n, mask, A, out);
}

void launch_ingest(int n, const double *src, int P, int64_t plane, double *A64, float *A32, int *flag, int *sym64,
                   int *symc, hipStream_t st)
{
    k_flags_init<<<1, 1, 0, st>>>(sym64, symc);
    dim3 blk(64, 4);
    k_ingest<<<node_grid(n, blk), blk, 0, st>>>(n, src, P, plane, A64, A32, flag, sym64, symc);
}

void launch_validate(int n, int P, int64_t plane, const double *A, int *flag, hipStream_t st)
{
    dim3 blk(64, 4);
    k_validate<<<node_grid(n, blk), blk, 0, st>>>(n, P, plane, A, flag);
}

}  // namespace mg
