// V-cycle kernels (Algorithm 1 in correction form) for a size class of
// (problem, level) slots:
//   outer residual r = f - A u in FP64 with per-block sums of squares,
//   convergence check (section 6.1 stopping rule), u += e,
//   first smoothing sweep from e = 0, residual s = r - A e, smoother
//   application e += M^{-1} s (damped Jacobi M = D/omega, section 2.1, or the
//   learned per-point 5x5 gather stencil, section 4), residual fused with
//   full-weighting restriction, bilinear prolongation e += P e_c.
// T = float: the mixed-precision inner cycle (FP32 arithmetic, BF16 smoother);
// T = double: the FP64 parity cycle.  Bandwidth-bound: one thread per node,
// rows of 64..256 consecutive nodes per block for coalesced plane reads.
#include "common.hpp"
#include "launch.hpp"

namespace mg {

namespace {

constexpr int kThreads = 256;

struct RowTile {
    int bx, by;
};
inline RowTile row_tile(int n)
{
    const int bx = n > 128 ? 256 : (n > 64 ? 128 : 64);
    return {bx, kThreads / bx};
}
inline dim3 row_grid(int n, RowTile t, int nslots)
{
    return dim3((n + t.bx - 1) / t.bx, (n + t.by - 1) / t.by, nslots);
}

// y = sum_d A[d] x_{p+d} over the 3x3 stencil; neighbours off the grid count
// as zero.  Loads are unconditional (clamped to the node itself) and the value
// is selected afterwards, so that the compiler can issue them together.
template <typename PA, typename PX, typename Acc>
__device__ inline Acc apply3x3(PA A, int64_t plane, PX x, int n, int P, int i, int j)
{
    const int64_t p = (int64_t)j * P + i;
    Acc acc = 0;
#pragma unroll
    for (int c = 0; c < 9; ++c) {
        const int ii = i + c % 3 - 1, jj = j + c / 3 - 1;
        const bool ok = ii >= 0 && ii < n && jj >= 0 && jj < n;
        const Acc a = (Acc)A[c * plane + p];
        const Acc xv = (Acc)x[ok ? (int64_t)jj * P + ii : p];
        acc += a * (ok ? xv : (Acc)0);
    }
    return acc;
}

// apply3x3 for a symmetric stencil: the four entries to the neighbours below and to
// the left are read from those neighbours' mirrored planes (A[c](p) = A[8-c](p + d_c)),
// so that only planes 4..8 are read from memory; the same values, summed in the same
// order, as apply3x3.
template <typename PA, typename PX, typename Acc>
__device__ inline Acc apply3x3_sym(PA A, int64_t plane, PX x, int n, int P, int i, int j)
{
    const int64_t p = (int64_t)j * P + i;
    Acc acc = 0;
#pragma unroll
    for (int c = 0; c < 9; ++c) {
        const int ii = i + c % 3 - 1, jj = j + c / 3 - 1;
        const bool ok = ii >= 0 && ii < n && jj >= 0 && jj < n;
        const int64_t q = ok ? (int64_t)jj * P + ii : p;
        const Acc a = (Acc)(c < 4 ? A[(8 - c) * plane + q] : A[c * plane + p]);
        const Acc xv = (Acc)x[q];
        acc += a * (ok ? xv : (Acc)0);
    }
    return acc;
}

// (H x)_p with H stored as 25 planes of H = W / a_C.
template <typename PH, typename PX, typename Acc>
__device__ inline Acc apply5x5(PH H, int64_t plane, PX x, int n, int P, int i, int j)
{
    const int64_t p = (int64_t)j * P + i;
    Acc acc = 0;
#pragma unroll
    for (int k = 0; k < 25; ++k) {
        const int ii = i + k % 5 - 2, jj = j + k / 5 - 2;
        const bool ok = ii >= 0 && ii < n && jj >= 0 && jj < n;
        const Acc h = (Acc)h2f(H[k * plane + p]);
        const Acc xv = (Acc)x[ok ? (int64_t)jj * P + ii : p];
        acc += h * (ok ? xv : (Acc)0);
    }
    return acc;
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_outer_residual(const OuterSlot<T> *slots, const SolveState *state)
{
    __shared__ double red[kThreads / 64];
    const TileId tile = xcd_tile();
    const OuterSlot<T> s = slots[tile.z];
    if (!state[s.prob].active) return;
    const int i = tile.x * blockDim.x + threadIdx.x;
    const int j = tile.y * blockDim.y + threadIdx.y;
    double r = 0.0;
    if (i < s.n && j < s.n) {
        const int64_t p = (int64_t)j * s.P + i;
        r = s.f[p] - (*s.sym ? apply3x3_sym<decltype(s.A64), decltype(s.u), double>(s.A64, s.plane, s.u, s.n, s.P, i, j)
                             : apply3x3<decltype(s.A64), decltype(s.u), double>(s.A64, s.plane, s.u, s.n, s.P, i, j));
        s.r[p] = (T)r;
    }
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    const double sum = block_sum<kThreads>(r * r, red);
    if (tid == 0) s.partial[tile.y * gridDim.x + tile.x] = sum;
}

// Tiles of node pairs for the outer residual on large grids: 32 threads cover 64 columns, 8 rows (the
// rows above a tile, read for its top row, come from L2 more often than with 4 rows: at n = 4095 the
// fetched bytes fall from 1.22 to 1.18 times the algorithmic ones, the time stays; 16 x 16 was slower).
constexpr int kPairResidualMin = 2047;  // below, one node per thread was faster (cache-resident grids)
inline RowTile pair_tile(int) { return {32, kThreads / 32}; }
inline dim3 pair_grid(int n, RowTile t, int nslots)
{
    return dim3(((n + 1) / 2 + t.bx - 1) / t.bx, (n + t.by - 1) / t.by, nslots);
}

// k_outer_residual on pairs of horizontally adjacent nodes (i, i+1), i even,
// one pair per thread, for n >= kPairResidualMin: stencil planes, u and f
// load as 16-byte words (a pair's right node may be the zero padding column).
// Each node's nine terms are summed in stencil order, as apply3x3 does.  For
// a symmetric stencil (OuterSlot::sym) only planes 4..8 are read: the entries
// to the row below and the left neighbour come from those neighbours'
// mirrored planes (stencil_index), pairs that start one column off.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_outer_residual_pairs(const OuterSlot<T> *slots, const SolveState *state)
{
    typedef double D2 __attribute__((ext_vector_type(2)));
    typedef double D2u __attribute__((ext_vector_type(2), aligned(8)));
    typedef T T2 __attribute__((ext_vector_type(2)));
    __shared__ double red[kThreads / 64];
    const TileId tile = xcd_tile();
    const OuterSlot<T> s = slots[tile.z];
    if (!state[s.prob].active) return;
    const int n = s.n, P = s.P;
    const int i = 2 * (tile.x * blockDim.x + threadIdx.x);
    const int j = tile.y * blockDim.y + threadIdx.y;
    const bool on = i < n && j < n;  // the pair's left node is on the grid
    const int64_t p = on ? (int64_t)j * P + i : 0;
    const bool sym = *s.sym != 0;
    // every load first, unconditionally (clamped addresses, values selected afterwards)
    D2 a[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) a[c] = *(const D2u MG_G *)(s.A64 + stencil_index(c, sym, s.plane, P, p));
    D2 uv[3][3];  // u pairs at columns i-2, i, i+2 of rows j-1 .. j+1 (zero off the grid)
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int row = j + dy - 1, col = i + 2 * k - 2;
            const bool ok = on && row >= 0 && row < n && col >= 0 && col < n;
            const D2 v = *(const D2 MG_G *)(s.u + (ok ? (int64_t)row * P + col : p));
            uv[dy][k] = ok ? v : D2{0.0, 0.0};
        }
    }
    const D2 fv = *(const D2 MG_G *)(s.f + p);
    double r0 = 0.0, r1 = 0.0;
    if (on) {
        double acc0 = 0.0, acc1 = 0.0;
#pragma unroll
        for (int c = 0; c < 9; ++c) {
            const int dy = c / 3, dx = c % 3;  // neighbour (i + dx - 1, j + dy - 1)
            const double x0 = dx == 0 ? uv[dy][0].y : dx == 1 ? uv[dy][1].x : uv[dy][1].y;
            const double x1 = dx == 0 ? uv[dy][1].x : dx == 1 ? uv[dy][1].y : uv[dy][2].x;
            acc0 += a[c].x * x0;
            acc1 += a[c].y * x1;
        }
        r0 = fv.x - acc0;
        r1 = i + 1 < n ? fv.y - acc1 : 0.0;
        T2 rv;
        rv.x = (T)r0;
        rv.y = (T)r1;
        *(T2 MG_G *)(s.r + p) = rv;
    }
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    const double sum = block_sum<kThreads>(r0 * r0 + r1 * r1, red);
    if (tid == 0) s.partial[tile.y * gridDim.x + tile.x] = sum;
}

// One block per slot.  init = 1: the partial sums are ||f||^2 (u = 0); set up
// the problem's state.  init = 0: the stopping rule of the solver.
template <typename T>
__global__ void __launch_bounds__(kThreads)
    k_check(const OuterSlot<T> *slots, SolveState *state, const SolveParams *prm, int init)
{
    __shared__ double red[kThreads / 64];
    const OuterSlot<T> s = slots[blockIdx.x];
    SolveState &st = state[s.prob];
    if (!init && !st.active) return;
    // four independent partial sums per thread, so that its loads are in flight together
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    const int np = st.nparts;
    int q = threadIdx.x;
    for (; q + 3 * kThreads < np; q += 4 * kThreads) {
        a0 += s.partial[q];
        a1 += s.partial[q + kThreads];
        a2 += s.partial[q + 2 * kThreads];
        a3 += s.partial[q + 3 * kThreads];
    }
    for (; q < np; q += kThreads) a0 += s.partial[q];
    const double rr = block_sum<kThreads>((a0 + a1) + (a2 + a3), red);
    if (threadIdx.x != 0) return;
    if (init) {
        st.fnorm = sqrt(rr);
        st.iters = 0;
        st.status = 0;
        st.active = 1;
        st.relres = 1.0;
        st.best = 1.0;
        st.stall = 0;
        st.fallback = 0;
        return;
    }
    stopping_rule(st, rr, prm, s.prob);
}

__global__ void k_sym_init(int *sym) { *sym = 1; }

template <typename T>
__global__ void __launch_bounds__(kThreads) k_sym_check(int n, int P, int64_t plane, const T *A, int *sym)
{
    const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (q >= (int64_t)n * n) return;
    const int i = (int)(q % n), j = (int)(q / n);
    const int64_t p = (int64_t)j * P + i;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int ii = i + c % 3 - 1, jj = j + c / 3 - 1;
        if (ii < 0 || ii >= n || jj < 0 || jj >= n) continue;
        if (!(A[c * plane + p] == A[(8 - c) * plane + (int64_t)jj * P + ii])) *sym = 0;  // every writer writes 0
    }
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_update_u(const OuterSlot<T> *slots, const SolveState *state)
{
    const OuterSlot<T> s = slots[blockIdx.z];
    if (!state[s.prob].active) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= s.n || j >= s.n) return;
    const int64_t p = (int64_t)j * s.P + i;
    s.u[p] += (double)s.e[p];
}

// First sweep from e = 0: e = M^{-1} r.
template <typename T, bool CNN>
__global__ void __launch_bounds__(kThreads) k_smooth_first(const CycleSlot<T> *slots, const SolveState *state, T omega)
{
    const CycleSlot<T> s = slots[blockIdx.z];
    if (!state[s.prob].active) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= s.n || j >= s.n) return;
    const int64_t p = (int64_t)j * s.P + i;
    T v;
    if (CNN)
        v = apply5x5<decltype(s.H), decltype(s.r), T>(s.H, s.plane, s.r, s.n, s.P, i, j);
    else
        v = omega * s.r[p] / s.A[kCentre * s.plane + p];
    s.e[p] = v;
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_residual(const CycleSlot<T> *slots, const SolveState *state)
{
    const CycleSlot<T> s = slots[blockIdx.z];
    if (!state[s.prob].active) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= s.n || j >= s.n) return;
    const int64_t p = (int64_t)j * s.P + i;
    s.s[p] = s.r[p] - apply3x3<decltype(s.A), decltype(s.e), T>(s.A, s.plane, s.e, s.n, s.P, i, j);
}

// e += M^{-1} s (s = r - A e from k_residual).
template <typename T, bool CNN>
__global__ void __launch_bounds__(kThreads) k_smooth_apply(const CycleSlot<T> *slots, const SolveState *state, T omega)
{
    const CycleSlot<T> s = slots[blockIdx.z];
    if (!state[s.prob].active) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= s.n || j >= s.n) return;
    const int64_t p = (int64_t)j * s.P + i;
    T v;
    if (CNN)
        v = apply5x5<decltype(s.H), decltype(s.s), T>(s.H, s.plane, s.s, s.n, s.P, i, j);
    else
        v = omega * s.s[p] / s.A[kCentre * s.plane + p];
    s.e[p] += v;
}

// Residual s = r - A e on the fine nodes under a tile of coarse nodes (staged
// in LDS), then r_c(I) = sum_a w_R(a) s(2I+1+a), w_R = (1/16)[1 2 1; 2 4 2; 1 2 1].
constexpr int kRcX = 32, kRcY = 8;                   // coarse tile
constexpr int kRfX = 2 * kRcX + 1, kRfY = 2 * kRcY + 1;  // fine region

template <typename T>
__global__ void __launch_bounds__(kThreads) k_residual_restrict(const CycleSlot<T> *slots, const SolveState *state)
{
    __shared__ T sres[kRfY][kRfX];
    const CycleSlot<T> s = slots[blockIdx.z];
    if (!state[s.prob].active) return;
    const int I0 = blockIdx.x * kRcX, J0 = blockIdx.y * kRcY;
    const int x0 = 2 * I0, y0 = 2 * J0;  // fine node 2*I0 is the left neighbour of coarse I0's node
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    for (int q = tid; q < kRfX * kRfY; q += kThreads) {
        const int fx = x0 + q % kRfX, fy = y0 + q / kRfX;
        T v = 0;
        if (fx < s.n && fy < s.n) {
            const int64_t p = (int64_t)fy * s.P + fx;
            v = s.r[p] - apply3x3<decltype(s.A), decltype(s.e), T>(s.A, s.plane, s.e, s.n, s.P, fx, fy);
        }
        sres[q / kRfX][q % kRfX] = v;
    }
    __syncthreads();
    const int tx = tid % kRcX, ty = tid / kRcX;
    const int I = I0 + tx, J = J0 + ty;
    if (I >= s.nc || J >= s.nc) return;
    const int cx = 2 * tx + 1, cy = 2 * ty + 1;
    const T acc = (T)0.0625 * (sres[cy - 1][cx - 1] + sres[cy - 1][cx + 1] + sres[cy + 1][cx - 1] + sres[cy + 1][cx + 1]) +
                  (T)0.125 * (sres[cy - 1][cx] + sres[cy + 1][cx] + sres[cy][cx - 1] + sres[cy][cx + 1]) +
                  (T)0.25 * sres[cy][cx];
    s.rc[(int64_t)J * s.Pc + I] = acc;
}

// e += P e_c: fine node 2I+1 takes e_c(I); nodes between two coarse nodes take
// half of each; cell centres a quarter of each of four.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_prolong(const CycleSlot<T> *slots, const SolveState *state)
{
    const CycleSlot<T> s = slots[blockIdx.z];
    if (!state[s.prob].active) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= s.n || j >= s.n) return;
    // coarse neighbours: one on odd coordinates, two (weights 1/2) on even ones
    const int ia = (i & 1) ? (i - 1) >> 1 : (i >> 1) - 1, ib = (i & 1) ? ia : ia + 1;
    const int ja = (j & 1) ? (j - 1) >> 1 : (j >> 1) - 1, jb = (j & 1) ? ja : ja + 1;
    const T wx = (i & 1) ? (T)1 : (T)0.5, wy = (j & 1) ? (T)1 : (T)0.5;
    const bool oka = ia >= 0, okb = ib < s.nc, okj = ja >= 0, okk = jb < s.nc;
    const T c00 = s.ec[(okj && oka) ? (int64_t)ja * s.Pc + ia : 0];
    const T c01 = s.ec[(okj && okb) ? (int64_t)ja * s.Pc + ib : 0];
    const T c10 = s.ec[(okk && oka) ? (int64_t)jb * s.Pc + ia : 0];
    const T c11 = s.ec[(okk && okb) ? (int64_t)jb * s.Pc + ib : 0];
    const bool two_x = !(i & 1), two_y = !(j & 1);
    T acc = (okj && oka ? c00 : (T)0) + (two_x && okj && okb ? c01 : (T)0) + (two_y && okk && oka ? c10 : (T)0) +
            (two_x && two_y && okk && okb ? c11 : (T)0);
    acc *= wx * wy;
    s.e[(int64_t)j * s.P + i] += acc;
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_zero_e(const CycleSlot<T> *slots, const SolveState *state)
{
    const CycleSlot<T> s = slots[blockIdx.z];
    if (!state[s.prob].active) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= s.n || j >= s.n) return;
    s.e[(int64_t)j * s.P + i] = 0;
}

__global__ void k_activate(SolveState *state, int nprob)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nprob) state[p].active = 1;
}

__global__ void k_zero_f64(double *x, int64_t count)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < count) x[q] = 0.0;
}

}  // namespace

void launch_activate(SolveState *state, int nprob, hipStream_t st)
{
    k_activate<<<(nprob + 255) / 256, 256, 0, st>>>(state, nprob);
}

void launch_zero_f64(double *x, int64_t count, hipStream_t st)
{
    k_zero_f64<<<(unsigned)((count + 255) / 256), 256, 0, st>>>(x, count);
}

int outer_residual_parts(int n)
{
    const RowTile t = n >= kPairResidualMin ? pair_tile(n) : row_tile(n);
    const dim3 g = n >= kPairResidualMin ? pair_grid(n, t, 1) : row_grid(n, t, 1);
    return (int)(g.x * g.y);
}

template <typename T>
void launch_outer_residual(const OuterSlot<T> *slots, int nslots, int n, const SolveState *state, hipStream_t st)
{
    if (n >= kPairResidualMin) {
        const RowTile t = pair_tile(n);
        k_outer_residual_pairs<T><<<pair_grid(n, t, nslots), dim3(t.bx, t.by), 0, st>>>(slots, state);
    } else {
        const RowTile t = row_tile(n);
        k_outer_residual<T><<<row_grid(n, t, nslots), dim3(t.bx, t.by), 0, st>>>(slots, state);
    }
}

template <typename T>
void launch_check(const OuterSlot<T> *slots, int nslots, SolveState *state, const SolveParams *prm, int init,
                  hipStream_t st)
{
    k_check<T><<<nslots, kThreads, 0, st>>>(slots, state, prm, init);
}

template <typename T>
void launch_check_symmetric(int n, int P, int64_t plane, const T *A, int *sym, hipStream_t st)
{
    k_sym_init<<<1, 1, 0, st>>>(sym);
    k_sym_check<T><<<(unsigned)(((int64_t)n * n + kThreads - 1) / kThreads), kThreads, 0, st>>>(n, P, plane, A, sym);
}
template void launch_check_symmetric<float>(int, int, int64_t, const float *, int *, hipStream_t);
template void launch_check_symmetric<double>(int, int, int64_t, const double *, int *, hipStream_t);

template <typename T>
void launch_update_u(const OuterSlot<T> *slots, int nslots, int n, const SolveState *state, hipStream_t st)
{
    const RowTile t = row_tile(n);
    k_update_u<T><<<row_grid(n, t, nslots), dim3(t.bx, t.by), 0, st>>>(slots, state);
}

template <typename T>
void launch_smooth_first(const CycleSlot<T> *slots, int nslots, int n, bool cnn, double omega,
                         const SolveState *state, hipStream_t st)
{
    const RowTile t = row_tile(n);
    if (cnn)
        k_smooth_first<T, true><<<row_grid(n, t, nslots), dim3(t.bx, t.by), 0, st>>>(slots, state, (T)omega);
    else
        k_smooth_first<T, false><<<row_grid(n, t, nslots), dim3(t.bx, t.by), 0, st>>>(slots, state, (T)omega);
}

template <typename T>
void launch_residual(const CycleSlot<T> *slots, int nslots, int n, const SolveState *state, hipStream_t st)
{
    const RowTile t = row_tile(n);
    k_residual<T><<<row_grid(n, t, nslots), dim3(t.bx, t.by), 0, st>>>(slots, state);
}

template <typename T>
void launch_smooth_apply(const CycleSlot<T> *slots, int nslots, int n, bool cnn, double omega,
                         const SolveState *state, hipStream_t st)
{
    const RowTile t = row_tile(n);
    if (cnn)
        k_smooth_apply<T, true><<<row_grid(n, t, nslots), dim3(t.bx, t.by), 0, st>>>(slots, state, (T)omega);
    else
        k_smooth_apply<T, false><<<row_grid(n, t, nslots), dim3(t.bx, t.by), 0, st>>>(slots, state, (T)omega);
}

template <typename T>
void launch_residual_restrict(const CycleSlot<T> *slots, int nslots, int n, const SolveState *state,
                              hipStream_t st)
{
    const int nc = (n - 1) / 2;
    const dim3 g((nc + kRcX - 1) / kRcX, (nc + kRcY - 1) / kRcY, nslots);
    k_residual_restrict<T><<<g, dim3(kRcX, kRcY), 0, st>>>(slots, state);
}

template <typename T>
void launch_prolong(const CycleSlot<T> *slots, int nslots, int n, const SolveState *state, hipStream_t st)
{
    const RowTile t = row_tile(n);
    k_prolong<T><<<row_grid(n, t, nslots), dim3(t.bx, t.by), 0, st>>>(slots, state);
}

template <typename T>
void launch_zero_e(const CycleSlot<T> *slots, int nslots, int n, const SolveState *state, hipStream_t st)
{
    const RowTile t = row_tile(n);
    k_zero_e<T><<<row_grid(n, t, nslots), dim3(t.bx, t.by), 0, st>>>(slots, state);
}

#define MG_INSTANTIATE(T)                                                                                        \
    template void launch_outer_residual<T>(const OuterSlot<T> *, int, int, const SolveState *, hipStream_t);      \
    template void launch_check<T>(const OuterSlot<T> *, int, SolveState *, const SolveParams *, int, hipStream_t); \
    template void launch_update_u<T>(const OuterSlot<T> *, int, int, const SolveState *, hipStream_t);           \
    template void launch_smooth_first<T>(const CycleSlot<T> *, int, int, bool, double, const SolveState *,       \
                                         hipStream_t);                                                           \
    template void launch_residual<T>(const CycleSlot<T> *, int, int, const SolveState *, hipStream_t);           \
    template void launch_smooth_apply<T>(const CycleSlot<T> *, int, int, bool, double, const SolveState *,       \
                                         hipStream_t);                                                           \
    template void launch_residual_restrict<T>(const CycleSlot<T> *, int, int, const SolveState *, hipStream_t);  \
    template void launch_prolong<T>(const CycleSlot<T> *, int, int, const SolveState *, hipStream_t);            \
    template void launch_zero_e<T>(const CycleSlot<T> *, int, int, const SolveState *, hipStream_t);
MG_INSTANTIATE(float)
MG_INSTANTIATE(double)
#undef MG_INSTANTIATE

}  // namespace mg
