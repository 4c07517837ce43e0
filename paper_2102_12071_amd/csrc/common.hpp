// Shared device/host definitions of the mgcnn library (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// Pointers held in device-side tables (slot structs) are marked as global
// memory in the device compilation pass, so that loads through them compile to
// global (not flat) memory instructions; the host pass sees plain pointers of
// the same size.
#if defined(__HIP_DEVICE_COMPILE__)
#define MG_G __attribute__((address_space(1)))
#else
#define MG_G
#endif

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

// ------------------------------------------------------- workgroup order
// The dispatcher hands workgroups to the 8 XCDs round-robin in linear block
// order (x fastest, then y, then z), and each XCD has its own L2.  Tiled
// kernels renumber their blocks so that every XCD runs one contiguous run of
// tiles: neighbouring tiles, which read the same halo cache lines, then share
// an L2.  The renumbering is a bijection of [0, nblocks) for any grid.
constexpr int kNumXcd = 8;
struct TileId {
    int x, y, z;
};
__device__ inline TileId xcd_tile()
{
    const int gx = gridDim.x, gy = gridDim.y;
    const int nb = gx * gy * gridDim.z;
    const int b = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const int xcd = b % kNumXcd, local = b / kNumXcd;
    const int q = nb / kNumXcd, r = nb % kNumXcd;
    const int t = xcd * q + min(xcd, r) + local;
    return TileId{t % gx, (t / gx) % gy, t / (gx * gy)};
}

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

__device__ inline float h2f(bf16_t v) { return bf16_to_f32(v); }
__device__ inline double h2f(double v) { return v; }
template <typename P>
__device__ inline auto load_h(P p) { return h2f(*p); }
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
    const T MG_G *A;                                   // 9 planes
    const typename SmootherStore<T>::type MG_G *H;     // 25 planes (H = W / a_C) or null
    T MG_G *r;                                         // level vectors
    T MG_G *e;
    T MG_G *s;
    T MG_G *rc;                                        // next coarser level's r and e
    T MG_G *ec;
    int nc, Pc;
    double MG_G *u;                                    // finest level only: the fused ascent adds e to u
    const int MG_G *sym;                               // 1: A[c](p) = A[8-c](p + d_c) wherever both nodes are
                                                       // on the grid (set with the level's stencil)
};

// Index of stencil entry c of node p (row pitch P, plane stride plane).  With a
// symmetric stencil (CycleSlot::sym) the entries to the row below and to the left
// neighbour come from the mirrored plane at that neighbour, A[c](p) =
// A[8-c](p + d_c), so planes 0..3 are never read: the same values.  An entry
// that points off the grid multiplies a zero correction either way; its
// mirrored index stays inside the nine planes (planes 5..8, one row and one
// column out at most), at a finite entry or the zero padding.
__device__ inline int64_t stencil_index(int c, bool sym, int64_t plane, int P, int64_t p)
{
    return (c < 4 && sym) ? (8 - c) * plane + p + (int64_t)(c / 3 - 1) * P + (c % 3 - 1) : c * plane + p;
}

// Finest level of a problem: FP64 state and the outer residual.
template <typename T>
struct OuterSlot {
    int prob;
    int n, P;
    int64_t plane;
    const double MG_G *A64;  // 9 planes FP64
    double MG_G *u;          // solution, FP64
    const double MG_G *f;    // right-hand side, FP64
    T MG_G *r;               // level-0 inner right-hand side (the residual)
    const T MG_G *e;         // level-0 inner correction
    double MG_G *partial;    // per-block partial sums of squares
    const int MG_G *sym;     // 1: the FP64 stencil is symmetric, A[c](p) = A[8-c](p + d_c) wherever both
                             // nodes are on the grid (set at set-up and on a new stencil)
};

// Levels with n <= kBottomMax run inside one workgroup per problem (bottom.hip).
constexpr int kBottomMax = 31;
constexpr int kMaxBottomLevels = 5;  // 31, 15, 7, 3, 1

template <typename T>
struct BottomLevel {
    int n, P;
    int64_t plane;
    const T MG_G *A;                                // 9 planes
    const typename SmootherStore<T>::type MG_G *H;  // 25 planes or null (coarsest)
};

template <typename T>
struct BottomSlot {
    int prob;
    int nlev;                                  // levels from the top one down to the coarsest
    BottomLevel<T> lev[kMaxBottomLevels];
    const double MG_G *Ainv;                   // coarsest inverse
    const T MG_G *r_in;                        // top level right-hand side (pitch lev[0].P)
    T MG_G *e_out;                             // top level correction
    double MG_G *u;                            // when the top level is the finest of a fused cycle: u += e
    const double MG_G *partial;                // the outer residual's block sums (the stopping rule folded in)
};

// Per-problem solver state on the device.
struct SolveState {
    int active;      // 1 while the problem still iterates
    int iters;       // V-cycles applied
    int status;      // 0 running/converged, 1 not converged, -4 diverged, 2 paused for the fallback
    int nparts;      // number of partial sums of the outer residual
    double fnorm;    // ||f||_2
    double relres;   // last relative residual
    double best;     // smallest relative residual so far
    int stall;       // cycles since best last improved by kStallGain
    int fallback;    // 0 none; 1 requested (stalled), 3 requested (diverged); 2 switched to damped Jacobi
};

// Fallback of the learned smoother to damped Jacobi: a problem whose residual
// has not improved on its best by 0.1 % for kStallCycles cycles, or has grown
// to kDivergeFactor times its best, is paused and switched.
constexpr int kStallCycles = 16;
constexpr double kStallGain = 1e-3;
constexpr double kDivergeFactor = 1e2;

// Stopping-rule parameters of one mg_solve call (read by the check kernel so
// that a captured iteration graph does not depend on them).
struct SolveParams {
    double tol;
    int maxit;
    int hist_stride;
    double *history;  // [nprob][hist_stride] or null
    int fallback;     // 1: a stalled or diverging learned smoother requests the switch to damped Jacobi
};

// The stopping rule of the solver (section 6.1) for one problem, given
// rr = ||f - A u||^2; called by one thread.
__device__ inline void stopping_rule(SolveState &st, double rr, const SolveParams *prm, int prob)
{
    const double rel = st.fnorm > 0.0 ? sqrt(rr) / st.fnorm : 0.0;
    st.relres = rel;
    if (prm->history) prm->history[(int64_t)prob * prm->hist_stride + st.iters] = rel;
    if (rel < st.best * (1.0 - kStallGain)) {
        st.best = rel;
        st.stall = 0;
    } else {
        st.stall += 1;
    }
    const bool diverging = !isfinite(rel) || rel > kDivergeFactor * st.best;
    if (rel <= prm->tol) {
        st.active = 0;
        st.status = 0;
    } else if (prm->fallback && st.fallback == 0 && (diverging || st.stall >= kStallCycles) &&
               st.iters < prm->maxit) {
        // pause (no cycle is applied); the host switches the problem to damped Jacobi and resumes it
        st.active = 0;
        st.status = 2;
        st.fallback = diverging ? 3 : 1;
    } else if (!isfinite(rel) || rel > 1e3) {
        st.active = 0;
        st.status = -4;
    } else if (st.iters >= prm->maxit) {
        st.active = 0;
        st.status = 1;
    } else {
        st.iters += 1;
    }
}

}  // namespace mg
