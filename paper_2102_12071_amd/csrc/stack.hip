// Convolution-stack smoother (the constant-coefficient alpha-CNN of section 5,
// full coarsening):
//     H x = f5(f4(f3(f2(f1(x))))) + f6(x),
// every f_i a single-channel 3x3 cross-correlation with zero padding: each
// intermediate grid is zero outside the n x n interior.  Weights w[layer][ky][kx]
// (layer 0..4 = f1..f5, 5 = f6); tap (ky, kx) reads x at (j + ky - 1, i + kx - 1).
//
// Apply: one workgroup per 64 x 16 output tile stages x with a halo of five
// nodes in LDS, runs the five composed layers there (each on a region one node
// narrower per side than the last, ping-ponging between two LDS buffers) and
// adds f6(x) from the staged x.  HBM traffic per node is x once plus the halo
// (1.9x for this tile, mostly from L2) and y read (when accumulating) and written; the 77
// multiply-adds per node read their operands from LDS through three-row
// register windows.
//
// Training (FP64, Algorithm 2): one layer per launch over a batch of vectors,
// and the weight gradients as per-block sums in a fixed order.
#include "stack.hpp"

namespace mg {

namespace {

constexpr int kTX = 64, kTY = 16, kHalo = 5;
constexpr int kLW = kTX + 2 * kHalo, kLH = kTY + 2 * kHalo;  // staged region 74 x 26
constexpr int kLN = kLW * kLH;
constexpr int kST = 256;
constexpr int kRun = 8;  // rows per thread in a layer's column walk

__device__ inline bool on_grid(int n, int i, int j) { return i >= 0 && i < n && j >= 0 && j < n; }

// One output tile (tx, ty) of y (+)= H x.
template <typename T>
__device__ void stack_tile(const T MG_G *x, T MG_G *y, const T MG_G *w, int n, int P, bool acc, int tx, int ty,
                           T *b0, T *b1, T *b2)
{
    const int i0 = tx * kTX - kHalo, j0 = ty * kTY - kHalo;  // grid node of staged slot (0, 0)
    const int tid = threadIdx.x;
    for (int q = tid; q < kLN; q += kST) {
        const int gi = i0 + q % kLW, gj = j0 + q / kLW;
        b0[q] = on_grid(n, gi, gj) ? x[(int64_t)gj * P + gi] : (T)0;
    }
    __syncthreads();
    const T *src = b0;
    T *dst = b1;
    // Each layer: a thread walks down one column of the region for kRun rows,
    // keeping three rows of the previous layer in registers (3 LDS reads per
    // output instead of 9).  Unrolled over layers, so every region size is a
    // compile-time constant.
#pragma unroll
    for (int layer = 0; layer < 5; ++layer) {
        const int m = layer + 1;  // this layer is valid on [m, kLW - m) x [m, kLH - m)
        const int rw = kLW - 2 * m, rh = kLH - 2 * m, chunks = (rh + kRun - 1) / kRun;
        T k[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) k[t] = w[layer * 9 + t];
        for (int q = tid; q < rw * chunks; q += kST) {
            const int xx = m + q % rw, y0 = m + (q / rw) * kRun;
            const int y1 = min(y0 + kRun, kLH - m);
            const bool col_in = i0 + xx >= 0 && i0 + xx < n;
            // rows y0 - 1 and y0 of the previous layer, valid on [m - 1, kLW - m]
            const T *c = src + (y0 - 1) * kLW + (xx - 1);
            T a0 = c[0], a1 = c[1], a2 = c[2];
            T b0r = c[kLW], b1r = c[kLW + 1], b2r = c[kLW + 2];
#pragma unroll
            for (int r = 0; r < kRun; ++r) {
                const int yy = y0 + r;
                if (yy < y1) {
                    const T *cn = src + (yy + 1) * kLW + (xx - 1);
                    const T c0 = cn[0], c1 = cn[1], c2 = cn[2];
                    const T v = k[0] * a0 + k[1] * a1 + k[2] * a2 + k[3] * b0r + k[4] * b1r + k[5] * b2r +
                                k[6] * c0 + k[7] * c1 + k[8] * c2;
                    const int gj = j0 + yy;
                    dst[yy * kLW + xx] = col_in && gj >= 0 && gj < n ? v : (T)0;
                    a0 = b0r, a1 = b1r, a2 = b2r;
                    b0r = c0, b1r = c1, b2r = c2;
                }
            }
        }
        __syncthreads();
        src = dst;
        dst = dst == b1 ? b2 : b1;
    }
    // output: src holds f5(..f1(x)) on the tile; add f6(x) from the staged x, same column walk
    T k6[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) k6[t] = w[45 + t];
    constexpr int kOutChunks = (kTY + kRun - 1) / kRun;
    for (int q = tid; q < kTX * kOutChunks; q += kST) {
        const int xx = kHalo + q % kTX, y0 = kHalo + (q / kTX) * kRun;
        const int gi = i0 + xx;  // >= 0 on the output tile
        if (gi >= n) continue;
        // the run's old y values first: loads issued together, not each behind the previous store
        T yv[kRun];
#pragma unroll
        for (int r = 0; r < kRun; ++r) {
            const int gj = j0 + y0 + r;
            yv[r] = acc && y0 + r < kHalo + kTY && gj < n ? y[(int64_t)gj * P + gi] : (T)0;
        }
        const T *c = b0 + (y0 - 1) * kLW + (xx - 1);
        T a0 = c[0], a1 = c[1], a2 = c[2];
        T b0r = c[kLW], b1r = c[kLW + 1], b2r = c[kLW + 2];
#pragma unroll
        for (int r = 0; r < kRun; ++r) {
            const int yy = y0 + r, gj = j0 + yy;
            if (yy < kHalo + kTY && gj < n) {
                const T *cn = b0 + (yy + 1) * kLW + (xx - 1);
                const T c0 = cn[0], c1 = cn[1], c2 = cn[2];
                const T v = src[yy * kLW + xx] + k6[0] * a0 + k6[1] * a1 + k6[2] * a2 + k6[3] * b0r +
                            k6[4] * b1r + k6[5] * b2r + k6[6] * c0 + k6[7] * c1 + k6[8] * c2;
                y[(int64_t)gj * P + gi] = yv[r] + v;
                a0 = b0r, a1 = b1r, a2 = b2r;
                b0r = c0, b1r = c1, b2r = c2;
            }
        }
    }
}

// mode 0: e = H r (first sweep); 1: e += H s before the coarse correction;
// 2: e += H' s after it.  The slot's H points to the level's two weight sets
// (before, after).
template <typename T>
__global__ void __launch_bounds__(kST) k_stack_cycle(const CycleSlot<T> *slots, const SolveState *state, int mode)
{
    __shared__ T b0[kLN], b1[kLN], b2[kLN];
    const TileId t = xcd_tile();
    const CycleSlot<T> s = slots[t.z];
    if (!state[s.prob].active) return;  // uniform over the workgroup
    const T MG_G *w = (const T MG_G *)s.H + (mode == 2 ? kStackWeights : 0);
    stack_tile<T>(mode == 0 ? s.r : s.s, s.e, w, s.n, s.P, mode != 0, t.x, t.y, b0, b1, b2);
}

__global__ void __launch_bounds__(kST) k_stack_vecs(const double *x, double *y, int64_t vs, const double *w, int n,
                                                    int P, int acc, const int *active)
{
    __shared__ double b0[kLN], b1[kLN], b2[kLN];
    const TileId t = xcd_tile();
    if (active && !active[t.z]) return;
    stack_tile<double>((const double MG_G *)(x + t.z * vs), (double MG_G *)(y + t.z * vs), (const double MG_G *)w, n,
                       P, acc != 0, t.x, t.y, b0, b1, b2);
}

__global__ void __launch_bounds__(kST) k_stack_layer(const double *x, double *y, int64_t vs, const double *w, int flip,
                                                     int n, int P, const int *active)
{
    const int q = blockIdx.x * kST + threadIdx.x, z = blockIdx.z;
    if (q >= n * n || (active && !active[z])) return;
    const int i = q % n, j = q / n;
    const double *xv = x + z * vs;
    double v = 0.0;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int ii = i + t % 3 - 1, jj = j + t / 3 - 1;
        if (on_grid(n, ii, jj)) v += w[flip ? 8 - t : t] * xv[(int64_t)jj * P + ii];
    }
    y[z * vs + (int64_t)j * P + i] = v;
}

// part[z][block][9 L + t] += sum over this block's nodes p of g[L]_p x[L]_{p + off(t)}
__global__ void __launch_bounds__(kST) k_stack_wgrad(StackPairs pr, int64_t vs, int n, int P, const int *active,
                                                     double *part)
{
    __shared__ double red[kST / 64];
    const int z = blockIdx.z;
    if (active && !active[z]) return;  // uniform over the workgroup
    const int q = blockIdx.x * kST + threadIdx.x;
    const bool ok = q < n * n;
    const int i = ok ? q % n : 0, j = ok ? q / n : 0;
    const int64_t o = z * vs;
    double *out = part + ((int64_t)z * gridDim.x + blockIdx.x) * kStackWeights;
    for (int L = 0; L < 6; ++L) {
        const double g = ok ? pr.g[L][o + (int64_t)j * P + i] : 0.0;
        for (int t = 0; t < 9; ++t) {
            const int ii = i + t % 3 - 1, jj = j + t / 3 - 1;
            const double v = ok && on_grid(n, ii, jj) ? g * pr.x[L][o + (int64_t)jj * P + ii] : 0.0;
            const double s = block_sum<kST>(v, red);
            if (threadIdx.x == 0) out[L * 9 + t] += s;
        }
    }
}

__global__ void k_stack_gsum(const double *part, int64_t nrow, double *grad)
{
    const int j = threadIdx.x;
    if (j >= kStackWeights) return;
    double s = 0.0;
    for (int64_t r = 0; r < nrow; ++r) s += part[r * kStackWeights + j];
    grad[j] = s;
}

// H^T = f1^T(f2^T(..f5^T)) + f6^T: the composed layers in reverse order, every
// kernel turned by 180 degrees
__global__ void k_stack_transpose(const double *w, double *wT)
{
    const int j = threadIdx.x;
    if (j >= kStackWeights) return;
    const int L = j / 9, t = j % 9;
    wT[j] = w[(L < 5 ? 4 - L : 5) * 9 + 8 - t];
}

__global__ void k_stack_adam(double *w, double *m, double *v, const double *g, int t, double lr, double b1, double b2,
                             double eps)
{
    const int j = threadIdx.x;
    if (j >= kStackWeights) return;
    m[j] = b1 * m[j] + (1.0 - b1) * g[j];
    v[j] = b2 * v[j] + (1.0 - b2) * g[j] * g[j];
    const double mh = m[j] / (1.0 - pow(b1, (double)t)), vh = v[j] / (1.0 - pow(b2, (double)t));
    w[j] -= lr * mh / (sqrt(vh) + eps);
}

inline dim3 tile_grid(int n, int count)
{
    return dim3((unsigned)((n + kTX - 1) / kTX), (unsigned)((n + kTY - 1) / kTY), (unsigned)count);
}

inline dim3 node_grid(int n, int count) { return dim3((unsigned)(((int64_t)n * n + kST - 1) / kST), 1, count); }

}  // namespace

template <typename T>
void launch_stack_cycle(const CycleSlot<T> *slots, int nslots, int n, int mode, const SolveState *state,
                        hipStream_t st)
{
    k_stack_cycle<T><<<tile_grid(n, nslots), kST, 0, st>>>(slots, state, mode);
}
template void launch_stack_cycle<float>(const CycleSlot<float> *, int, int, int, const SolveState *, hipStream_t);
template void launch_stack_cycle<double>(const CycleSlot<double> *, int, int, int, const SolveState *, hipStream_t);

void launch_stack_vecs(const double *x, double *y, int64_t vs, const double *w, int n, int P, int count,
                       bool accumulate, const int *active, hipStream_t st)
{
    k_stack_vecs<<<tile_grid(n, count), kST, 0, st>>>(x, y, vs, w, n, P, accumulate ? 1 : 0, active);
}

void launch_stack_layer(const double *x, double *y, int64_t vs, const double *w, bool flip, int n, int P, int count,
                        const int *active, hipStream_t st)
{
    k_stack_layer<<<node_grid(n, count), kST, 0, st>>>(x, y, vs, w, flip ? 1 : 0, n, P, active);
}

int stack_wgrad_blocks(int n) { return (int)(((int64_t)n * n + kST - 1) / kST); }

void launch_stack_wgrad(const StackPairs &pr, int64_t vs, int n, int P, int count, const int *active, double *part,
                        hipStream_t st)
{
    k_stack_wgrad<<<node_grid(n, count), kST, 0, st>>>(pr, vs, n, P, active, part);
}

void launch_stack_gsum(const double *part, int64_t nrow, double *grad, hipStream_t st)
{
    k_stack_gsum<<<1, 64, 0, st>>>(part, nrow, grad);
}

void launch_stack_transpose(const double *w, double *wT, hipStream_t st) { k_stack_transpose<<<1, 64, 0, st>>>(w, wT); }

void launch_stack_adam(double *w, double *m, double *v, const double *g, int t, double lr, double b1, double b2,
                       double eps, hipStream_t st)
{
    k_stack_adam<<<1, 64, 0, st>>>(w, m, v, g, t, lr, b1, b2, eps);
}

}  // namespace mg
