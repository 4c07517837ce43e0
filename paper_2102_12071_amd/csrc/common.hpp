// Shared device/host definitions of the mgcnn library (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mg {

// ---------------------------------------------------------------- constants
constexpr int kStencil = 9;    // 3x3 operator stencil, channel 3(dy+1)+(dx+1)
constexpr int kSmoother = 25;  // 5x5 smoother stencil, channel 5(dy+2)+(dx+2)
constexpr int kCentre = 4;     // centre channel of the operator stencil
constexpr int kMaxLevels = 14;
constexpr int kMaxCoarseUnknowns = 49;  // coarsest grid up to 7 x 7

// A grid vector on a level: rows of pitch P = n + 1 elements (a power of two
// for n = 2^k - 1, so rows start aligned); element (i, j) at j*P + i.  The
// column i = n is padding and stays zero.  A field of C channels stores C
// such planes, plane stride n*P.
__host__ __device__ inline int64_t plane_of(int n, int P) { return (int64_t)n * P; }

// ------------------------------------------------------------------- bf16
// Storage as raw 16-bit words; conversion is round-to-nearest-even (the
// hardware v_cvt_pk_bf16_f32 on gfx950).
typedef uint16_t bf16_t;
__device__ inline float bf16_to_f32(bf16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
__device__ inline bf16_t f32_to_bf16(float f)
{
    __bf16 b = (__bf16)f;
    return __builtin_bit_cast(bf16_t, b);
}

// Smoother storage type per compute type: BF16 for the FP32 (mixed) cycle,
// FP64 for the FP64 parity cycle.
template <typename T> struct SmootherStore;
template <> struct SmootherStore<float> { typedef bf16_t type; };
template <> struct SmootherStore<double> { typedef double type; };

__device__ inline float load_h(const bf16_t *p) { return bf16_to_f32(*p); }
__device__ inline double load_h(const double *p) { return *p; }
__device__ inline void store_h(bf16_t *p, float v) { *p = f32_to_bf16(v); }
__device__ inline void store_h(double *p, double v) { *p = v; }

// ------------------------------------------------------------ reductions
// 64-lane wavefront sum, then across the waves of a block through LDS.
// Deterministic for a fixed block shape.
__device__ inline double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Waves are formed from the linear thread index (x fastest).
template <int NT>
__device__ inline double block_sum(double v, double *lds /* >= NT/64 */)
{
    v = wave_sum(v);
    const int tid = (threadIdx.z * blockDim.y + threadIdx.y) * blockDim.x + threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    __syncthreads();
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (tid == 0) {
        for (int w = 0; w < NT / 64; ++w) s += lds[w];
    }
    return s;  // valid in thread 0
}

// ------------------------------------------------------------------ slots
// One (problem, level) pair of a size class.  Every slot of a class has the
// same n, so one launch covers the class with blockIdx.z = slot.
template <typename T>
struct CycleSlot {
    int prob;
    int n, P;
    int64_t plane;
    const T *A;                                   // 9 planes
    const typename SmootherStore<T>::type *H;     // 25 planes (H = W / a_C) or null
    T *r, *e, *s;                                 // level vectors
    T *rc, *ec;                                   // next coarser level's r and e
    int nc, Pc;
};

// Finest level of a problem: FP64 state and the outer residual.
template <typename T>
struct OuterSlot {
    int prob;
    int n, P;
    int64_t plane;
    const double *A64;  // 9 planes FP64
    double *u;          // solution, FP64
    const double *f;    // right-hand side, FP64
    T *r;               // level-0 inner right-hand side (the residual)
    const T *e;         // level-0 inner correction
    double *partial;    // per-block partial sums of squares
};

// Coarsest level: explicit inverse of the (m*m) x (m*m) matrix.
template <typename T>
struct CoarseSlot {
    int prob;
    int m, P;
    const double *Ainv;  // [m*m][m*m] row-major, FP64
    const T *r;
    T *e;
};

// Per-problem solver state on the device.
struct SolveState {
    int active;      // 1 while the problem still iterates
    int iters;       // V-cycles applied
    int status;      // 0 running/converged, 1 not converged, -4 diverged
    int nparts;      // number of partial sums of the outer residual
    double fnorm;    // ||f||_2
    double relres;   // last relative residual
};

// Stopping-rule parameters of one mg_solve call (read by the check kernel so
// that a captured iteration graph does not depend on them).
struct SolveParams {
    double tol;
    int maxit;
    int hist_stride;
    double *history;  // [nprob][hist_stride] or null
};

}  // namespace mg
