// Coarsest-level direct solve (Algorithm 1: "solve A u = r" on the last
// level).  At setup one workgroup assembles the dense matrix of the coarsest
// stencil (at most 49 x 49), factors it by Cholesky in LDS and forms the
// explicit inverse column by column; every cycle then applies the inverse as
// a small dense FP64 product inside the bottom-levels kernel.
#include "common.hpp"
#include "launch.hpp"

namespace mg {

namespace {

constexpr int kN = kMaxCoarseUnknowns;

// One workgroup of kCT threads; every step's work is spread over all of them (right-looking forms):
// the factor subtracts the same products in the same order as the dot-product form L[i][k] = (A[i][k]
// - sum_{q<k} L[i][q] L[k][q]) / L[k][k], and the forward substitution likewise; the backward one
// subtracts the later rows' terms from the last row down.
constexpr int kCT = 256;
__global__ void __launch_bounds__(kCT) k_coarse_factor(int m, int P, int64_t plane, const double *A, double *Ainv,
                                                       int *flag)
{
    __shared__ double L[kN][kN + 1];  // the matrix, overwritten by its Cholesky factor (lower triangle)
    __shared__ double X[kN][kN + 1];
    __shared__ int bad;
    const int mm = m * m;
    const int t = threadIdx.x;
    if (t == 0) bad = 0;
    for (int q = t; q < mm * mm; q += kCT) {
        L[q / mm][q % mm] = 0.0;
        X[q / mm][q % mm] = q / mm == q % mm ? 1.0 : 0.0;
    }
    __syncthreads();
    // dense matrix: row p = j*m + i, column of the neighbour (i+dx, j+dy)
    for (int p = t; p < mm; p += kCT) {
        const int i = p % m, j = p / m;
        for (int c = 0; c < 9; ++c) {
            const int ii = i + c % 3 - 1, jj = j + c / 3 - 1;
            if (ii < 0 || ii >= m || jj < 0 || jj >= m) continue;
            L[p][jj * m + ii] = A[c * plane + (int64_t)j * P + i];
        }
    }
    __syncthreads();
    // Cholesky: column k is final once the updates of columns 0 .. k-1 are in
    for (int k = 0; k < mm; ++k) {
        if (t == 0) {
            double d = L[k][k];
            if (!(d > 0.0)) {
                bad = 1;
                d = 1.0;
            }
            L[k][k] = sqrt(d);
        }
        __syncthreads();
        for (int i = k + 1 + t; i < mm; i += kCT) L[i][k] /= L[k][k];
        __syncthreads();
        const int r = mm - k - 1;  // trailing block, lower triangle: L[i][j] -= L[i][k] L[j][k], k < j <= i
        for (int q = t; q < r * r; q += kCT) {
            const int i = k + 1 + q / r, j = k + 1 + q % r;
            if (j <= i) L[i][j] -= L[i][k] * L[j][k];
        }
        __syncthreads();
    }
    // inverse, all columns at once: L Y = I (rows in increasing order), then L^T X = Y (decreasing)
    for (int q = 0; q < mm; ++q) {
        for (int c = t; c < mm; c += kCT) X[q][c] /= L[q][q];
        __syncthreads();
        const int r = mm - q - 1;
        for (int e = t; e < r * mm; e += kCT) {
            const int i = q + 1 + e / mm, c = e % mm;
            X[i][c] -= L[i][q] * X[q][c];
        }
        __syncthreads();
    }
    for (int q = mm - 1; q >= 0; --q) {
        for (int c = t; c < mm; c += kCT) X[q][c] /= L[q][q];
        __syncthreads();
        for (int e = t; e < q * mm; e += kCT) {
            const int i = e / mm, c = e % mm;
            X[i][c] -= L[q][i] * X[q][c];
        }
        __syncthreads();
    }
    for (int q = t; q < mm * mm; q += kCT) Ainv[q] = X[q / mm][q % mm];
    if (t == 0 && bad) atomicOr(flag, 8);
}

}  // namespace

void launch_coarse_factor(int m, int P, int64_t plane, const double *A, double *Ainv, int *flag, hipStream_t st)
{
    k_coarse_factor<<<1, kCT, 0, st>>>(m, P, plane, A, Ainv, flag);
}

}  // namespace mg
