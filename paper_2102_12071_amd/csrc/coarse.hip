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

__global__ void __launch_bounds__(64) k_coarse_factor(int m, int P, int64_t plane, const double *A, double *Ainv,
                                                      int *flag)
{
    __shared__ double L[kN][kN + 1];
    __shared__ double X[kN][kN + 1];
    __shared__ int bad;
    const int mm = m * m;
    const int t = threadIdx.x;
    if (t == 0) bad = 0;
    for (int q = t; q < mm * mm; q += 64) L[q / mm][q % mm] = 0.0;
    __syncthreads();
    // dense matrix: row p = j*m + i, column of the neighbour (i+dx, j+dy)
    for (int p = t; p < mm; p += 64) {
        const int i = p % m, j = p / m;
        for (int c = 0; c < 9; ++c) {
            const int ii = i + c % 3 - 1, jj = j + c / 3 - 1;
            if (ii < 0 || ii >= m || jj < 0 || jj >= m) continue;
            L[p][jj * m + ii] = A[c * plane + (int64_t)j * P + i];
        }
    }
    __syncthreads();
    // Cholesky, column by column: L[k][k] then the entries below it
    for (int k = 0; k < mm; ++k) {
        if (t == 0) {
            double d = L[k][k];
            for (int q = 0; q < k; ++q) d -= L[k][q] * L[k][q];
            if (!(d > 0.0)) {
                bad = 1;
                d = 1.0;
            }
            L[k][k] = sqrt(d);
        }
        __syncthreads();
        for (int i = k + 1 + t; i < mm; i += 64) {
            double s = L[i][k];
            for (int q = 0; q < k; ++q) s -= L[i][q] * L[k][q];
            L[i][k] = s / L[k][k];
        }
        __syncthreads();
    }
    // inverse: thread c solves L L^T x = e_c
    for (int c = t; c < mm; c += 64) {
        for (int i = 0; i < mm; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int q = 0; q < i; ++q) s -= L[i][q] * X[q][c];
            X[i][c] = s / L[i][i];
        }
        for (int i = mm - 1; i >= 0; --i) {
            double s = X[i][c];
            for (int q = i + 1; q < mm; ++q) s -= L[q][i] * X[q][c];
            X[i][c] = s / L[i][i];
        }
    }
    __syncthreads();
    for (int q = t; q < mm * mm; q += 64) Ainv[q] = X[q / mm][q % mm];
    if (t == 0 && bad) atomicOr(flag, 8);
}

}  // namespace

void launch_coarse_factor(int m, int P, int64_t plane, const double *A, double *Ainv, int *flag, hipStream_t st)
{
    k_coarse_factor<<<1, 64, 0, st>>>(m, P, plane, A, Ainv, flag);
}

}  // namespace mg
