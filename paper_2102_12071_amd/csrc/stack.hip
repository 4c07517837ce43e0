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

// The five composed layers f5(..f1(x)) on a staged W x Hh region whose slot (0, 0)
// is grid node (i0, j0): x in b0 (zero off the grid); layer L is computed on the
// region one node narrower per side than layer L - 1, ping-ponging between b1
// and b2.  Returns the buffer holding the result, valid on [5, W - 5) x [5, Hh - 5).
// Each layer: a thread walks down one column of the region for kRun rows, keeping
// three rows of the previous layer in registers (3 LDS reads per output instead
// of 9).  Unrolled over layers, so every region size is a compile-time constant.
template <typename T, int W, int Hh, int NT = kST>
__device__ const T *stack_layers(const T *b0, T *b1, T *b2, const T MG_G *w, int i0, int j0, int n)
{
    const int tid = threadIdx.x;
    const T *src = b0;
    T *dst = b1;
#pragma unroll
    for (int layer = 0; layer < 5; ++layer) {
        const int m = layer + 1;  // this layer is valid on [m, W - m) x [m, Hh - m)
        const int rw = W - 2 * m, rh = Hh - 2 * m, chunks = (rh + kRun - 1) / kRun;
        T k[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) k[t] = w[layer * 9 + t];
        for (int q = tid; q < rw * chunks; q += NT) {
            const int xx = m + q % rw, y0 = m + (q / rw) * kRun;
            const int y1 = min(y0 + kRun, Hh - m);
            const bool col_in = i0 + xx >= 0 && i0 + xx < n;
            // rows y0 - 1 and y0 of the previous layer, valid on [m - 1, W - m]
            const T *c = src + (y0 - 1) * W + (xx - 1);
            T a0 = c[0], a1 = c[1], a2 = c[2];
            T b0r = c[W], b1r = c[W + 1], b2r = c[W + 2];
#pragma unroll
            for (int r = 0; r < kRun; ++r) {
                const int yy = y0 + r;
                if (yy < y1) {
                    const T *cn = src + (yy + 1) * W + (xx - 1);
                    const T c0 = cn[0], c1 = cn[1], c2 = cn[2];
                    const T v = k[0] * a0 + k[1] * a1 + k[2] * a2 + k[3] * b0r + k[4] * b1r + k[5] * b2r +
                                k[6] * c0 + k[7] * c1 + k[8] * c2;
                    const int gj = j0 + yy;
                    dst[yy * W + xx] = col_in && gj >= 0 && gj < n ? v : (T)0;
                    a0 = b0r, a1 = b1r, a2 = b2r;
                    b0r = c0, b1r = c1, b2r = c2;
                }
            }
        }
        __syncthreads();
        src = dst;
        dst = dst == b1 ? b2 : b1;
    }
    return src;
}

// f6(x) at region slot (xx, yy) of a staged W-wide region, plus the layers' value lv
// (the sum in the order of the column walks above).
template <typename T, int W>
__device__ inline T stack_out(const T *b0, const T (&k6)[9], T lv, int xx, int yy)
{
    const T *c = b0 + (yy - 1) * W + (xx - 1);
    return lv + k6[0] * c[0] + k6[1] * c[1] + k6[2] * c[2] + k6[3] * c[W] + k6[4] * c[W + 1] + k6[5] * c[W + 2] +
           k6[6] * c[2 * W] + k6[7] * c[2 * W + 1] + k6[8] * c[2 * W + 2];
}

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
    const T *src = stack_layers<T, kLW, kLH>(b0, b1, b2, w, i0, j0, n);
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

// Fused level kernels of the V(1,1) cycle with the stack smoother (the same steps,
// in the same arithmetic, as the step kernels: stack sweep, residual and
// restriction going down; prolongation, residual and stack sweep coming up), so
// that the intermediate vectors stay in LDS and each level takes one launch per
// direction.  Regions are staged with the halos the next step needs (the stack
// reaches kHalo = 5 nodes, the stencil 1); neighbouring workgroups recompute the
// shared halos.
//
// Descend, per tile of kSDX x kSDY coarse nodes:
//   e = H r on the fine nodes the residual needs (the restriction's 2 kSDX + 1
//   columns plus one on each side), from r staged with 5 more; e written for the
//   fine nodes the tile owns; s = r - A e; r_c = R s (full weighting).
constexpr int kSDX = 32, kSDY = 8;
constexpr int kSSW = 2 * kSDX + 1, kSSH = 2 * kSDY + 1;        // residual region
constexpr int kSEW = kSSW + 2, kSEH = kSSH + 2;                // e region
constexpr int kSRW = kSEW + 2 * kHalo, kSRH = kSEH + 2 * kHalo;  // staged r
static_assert(kSDX * kSDY <= kST, "one thread per coarse node of the tile");

// NT threads: kST on large grids, more on the small ones, where a few workgroups run alone and
// the length of each step (nodes per thread) sets the time
template <typename T, int NT>
__global__ void __launch_bounds__(NT) k_stack_descend(const CycleSlot<T> *slots, const SolveState *state)
{
    __shared__ T b0[kSRW * kSRH], b1[kSRW * kSRH], b2[kSRW * kSRH];
    __shared__ T eb[kSEW * kSEH];
    __shared__ T sb[kSSW * kSSH];
    const TileId t = xcd_tile();
    const CycleSlot<T> s = slots[t.z];
    if (!state[s.prob].active) return;  // uniform over the workgroup
    const bool sym = *s.sym != 0;
    const int n = s.n, nc = s.nc, P = s.P, tid = threadIdx.x;
    const int I0 = t.x * kSDX, J0 = t.y * kSDY;
    const int sx0 = 2 * I0, sy0 = 2 * J0;           // residual region origin
    const int ex0 = sx0 - 1, ey0 = sy0 - 1;         // e region origin
    const int rx0 = ex0 - kHalo, ry0 = ey0 - kHalo;  // staged r origin
    const int ox1 = (I0 + kSDX >= nc) ? n : sx0 + 2 * kSDX;  // owned fine nodes [sx0, ox1) x [sy0, oy1)
    const int oy1 = (J0 + kSDY >= nc) ? n : sy0 + 2 * kSDY;
    const T MG_G *w = (const T MG_G *)s.H;
    // every global operand first (the stencil too in FP32), so that the workgroup waits for memory once
    constexpr int NRQ = (kSRW * kSRH + NT - 1) / NT, NSQ = (kSSW * kSSH + NT - 1) / NT;
    constexpr bool PA = sizeof(T) == 4;
    T rq[NRQ], aq[PA ? NSQ : 1][9];
#pragma unroll
    for (int k = 0; k < NRQ; ++k) {
        const int q = tid + k * NT;
        const int gi = rx0 + q % kSRW, gj = ry0 + q / kSRW;
        const bool ok = q < kSRW * kSRH && on_grid(n, gi, gj);
        const T v = s.r[ok ? (int64_t)gj * P + gi : 0];
        rq[k] = ok ? v : (T)0;
    }
    if (PA) {
#pragma unroll
        for (int k = 0; k < NSQ; ++k) {
            const int q = tid + k * NT;
            const int fx = sx0 + q % kSSW, fy = sy0 + q / kSSW;
            const int64_t p = q < kSSW * kSSH && fx < n && fy < n ? (int64_t)fy * P + fx : 0;
#pragma unroll
            for (int c = 0; c < 9; ++c) aq[PA ? k : 0][c] = s.A[stencil_index(c, sym, s.plane, P, p)];  // unused off the grid
        }
    }
#pragma unroll
    for (int k = 0; k < NRQ; ++k) {
        const int q = tid + k * NT;
        if (q < kSRW * kSRH) b0[q] = rq[k];
    }
    __syncthreads();
    const T *lay = stack_layers<T, kSRW, kSRH, NT>(b0, b1, b2, w, rx0, ry0, n);
    T k6[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) k6[k] = w[45 + k];
    for (int q = tid; q < kSEW * kSEH; q += NT) {
        const int x = q % kSEW, y = q / kSEW;
        const int gi = ex0 + x, gj = ey0 + y;
        T v = 0;
        if (on_grid(n, gi, gj)) {
            const int xx = x + kHalo, yy = y + kHalo;
            v = (T)0 + stack_out<T, kSRW>(b0, k6, lay[yy * kSRW + xx], xx, yy);  // e = 0 + H r
            if (gi >= sx0 && gi < ox1 && gj >= sy0 && gj < oy1) s.e[(int64_t)gj * P + gi] = v;
        }
        eb[q] = v;
    }
    __syncthreads();
    // s = r - A e (terms in the stencil's channel order)
#pragma unroll
    for (int k = 0; k < NSQ; ++k) {
        const int q = tid + k * NT;
        if (q >= kSSW * kSSH) break;
        const int x = q % kSSW, y = q / kSSW;
        const int fx = sx0 + x, fy = sy0 + y;
        T v = 0;
        if (fx < n && fy < n) {
            const int64_t p = (int64_t)fy * P + fx;
            T acc = 0;
#pragma unroll
            for (int c = 0; c < 9; ++c)
                acc += (PA ? aq[PA ? k : 0][c] : s.A[stencil_index(c, sym, s.plane, P, p)]) * eb[(y + c / 3) * kSEW + x + c % 3];
            v = b0[(y + 1 + kHalo) * kSRW + x + 1 + kHalo] - acc;
        }
        sb[q] = v;
    }
    __syncthreads();
    const int tx = tid % kSDX, ty = tid / kSDX;
    const int I = I0 + tx, J = J0 + ty;
    if (tid >= kSDX * kSDY || I >= nc || J >= nc) return;
    const int cx = 2 * tx + 1, cy = 2 * ty + 1;
    auto S = [&](int yy, int xx) { return sb[yy * kSSW + xx]; };
    const T acc = (T)0.0625 * (S(cy - 1, cx - 1) + S(cy - 1, cx + 1) + S(cy + 1, cx - 1) + S(cy + 1, cx + 1)) +
                  (T)0.125 * (S(cy - 1, cx) + S(cy + 1, cx) + S(cy, cx - 1) + S(cy, cx + 1)) + (T)0.25 * S(cy, cx);
    s.rc[(int64_t)J * s.Pc + I] = acc;
}

// Ascend, per tile of kSAX x kSAY fine nodes: e' = e + P e_c on the tile plus 6
// nodes, s = r - A e' on the tile plus 5, e = e' + H' s on the tile (the second
// weight set).  On the finest level the result is added to u; on the others it
// goes to s, where the next finer level's ascent reads it as e_c (e itself is
// still read by neighbouring tiles).
constexpr int kSAX = kTX, kSAY = kTY;
constexpr int kSAW = kLW, kSAH = kLH;                    // s region: the tile plus kHalo
constexpr int kSPW = kSAW + 2, kSPH = kSAH + 2;          // e' region
constexpr int kSCW = kSAX / 2 + 8, kSCH = kSAY / 2 + 8;  // coarse nodes under e'

template <typename T, bool PA, int NT>
__global__ void __launch_bounds__(NT) k_stack_ascend(const CycleSlot<T> *slots, const SolveState *state)
{
    __shared__ T cb[kSCW * kSCH];
    __shared__ T pb[kSPW * kSPH];
    __shared__ T b0[kLN], b1[kLN], b2[kLN];
    const TileId t = xcd_tile();
    const CycleSlot<T> s = slots[t.z];
    if (!state[s.prob].active) return;  // uniform over the workgroup
    const bool sym = *s.sym != 0;
    const int n = s.n, nc = s.nc, P = s.P, tid = threadIdx.x;
    const int X0 = t.x * kSAX, Y0 = t.y * kSAY;
    const int sx0 = X0 - kHalo, sy0 = Y0 - kHalo;  // s region origin
    const int px0 = sx0 - 1, py0 = sy0 - 1;        // e' region origin
    const int cx0 = X0 / 2 - 4, cy0 = Y0 / 2 - 4;  // coarse region origin
    const T MG_G *w = (const T MG_G *)s.H + kStackWeights;
    // every global operand first (with PA r and the stencil too), so that the workgroup waits for
    // memory once; without PA (large FP32 grids, where occupancy hides the latency, and FP64) r and
    // the stencil are read in the residual step
    constexpr int NCQ = (kSCW * kSCH + NT - 1) / NT, NPQ = (kSPW * kSPH + NT - 1) / NT;
    constexpr int NSQ = (kLN + NT - 1) / NT;
    T cq[NCQ], eq[NPQ], rq[PA ? NSQ : 1], aq[PA ? NSQ : 1][9];
#pragma unroll
    for (int k = 0; k < NCQ; ++k) {
        const int q = tid + k * NT;
        const int I = cx0 + q % kSCW, J = cy0 + q / kSCW;
        const bool ok = q < kSCW * kSCH && I >= 0 && I < nc && J >= 0 && J < nc;
        const T v = s.ec[ok ? (int64_t)J * s.Pc + I : 0];
        cq[k] = ok ? v : (T)0;
    }
#pragma unroll
    for (int k = 0; k < NPQ; ++k) {
        const int q = tid + k * NT;
        const int i = px0 + q % kSPW, j = py0 + q / kSPW;
        const bool ok = q < kSPW * kSPH && on_grid(n, i, j);
        const T v = s.e[ok ? (int64_t)j * P + i : 0];
        eq[k] = ok ? v : (T)0;
    }
    if (PA) {
#pragma unroll
        for (int k = 0; k < NSQ; ++k) {
            const int q = tid + k * NT;
            const int i = sx0 + q % kSAW, j = sy0 + q / kSAW;
            const int64_t p = q < kLN && on_grid(n, i, j) ? (int64_t)j * P + i : 0;
            rq[PA ? k : 0] = s.r[p];  // unused off the grid
#pragma unroll
            for (int c = 0; c < 9; ++c) aq[PA ? k : 0][c] = s.A[stencil_index(c, sym, s.plane, P, p)];
        }
    }
#pragma unroll
    for (int k = 0; k < NCQ; ++k) {
        const int q = tid + k * NT;
        if (q < kSCW * kSCH) cb[q] = cq[k];
    }
    __syncthreads();
    // e' = e + P e_c: fine node 2I+1 takes e_c(I); even nodes half of each neighbour
#pragma unroll
    for (int k = 0; k < NPQ; ++k) {
        const int q = tid + k * NT;
        if (q >= kSPW * kSPH) break;
        const int i = px0 + q % kSPW, j = py0 + q / kSPW;
        T v = 0;
        if (on_grid(n, i, j)) {
            const int ia = (i & 1) ? (i - 1) >> 1 : (i >> 1) - 1, ib = (i & 1) ? ia : ia + 1;
            const int ja = (j & 1) ? (j - 1) >> 1 : (j >> 1) - 1, jb = (j & 1) ? ja : ja + 1;
            const T wx = (i & 1) ? (T)1 : (T)0.5, wy = (j & 1) ? (T)1 : (T)0.5;
            const bool oka = ia >= 0, okb = ib < nc, okj = ja >= 0, okk = jb < nc;
            const T c00 = cb[(ja - cy0) * kSCW + ia - cx0], c01 = cb[(ja - cy0) * kSCW + ib - cx0];
            const T c10 = cb[(jb - cy0) * kSCW + ia - cx0], c11 = cb[(jb - cy0) * kSCW + ib - cx0];
            const bool two_x = !(i & 1), two_y = !(j & 1);
            T acc = (okj && oka ? c00 : (T)0) + (two_x && okj && okb ? c01 : (T)0) +
                    (two_y && okk && oka ? c10 : (T)0) + (two_x && two_y && okk && okb ? c11 : (T)0);
            acc *= wx * wy;
            v = eq[k] + acc;
        }
        pb[q] = v;
    }
    __syncthreads();
    // s = r - A e' (terms in the stencil's channel order), zero off the grid
#pragma unroll
    for (int k = 0; k < NSQ; ++k) {
        const int q = tid + k * NT;
        if (q >= kLN) break;
        const int x = q % kSAW, y = q / kSAW;
        const int i = sx0 + x, j = sy0 + y;
        T v = 0;
        if (on_grid(n, i, j)) {
            const int64_t p = (int64_t)j * P + i;
            T acc = 0;
#pragma unroll
            for (int c = 0; c < 9; ++c)
                acc += (PA ? aq[PA ? k : 0][c] : s.A[stencil_index(c, sym, s.plane, P, p)]) * pb[(y + c / 3) * kSPW + x + c % 3];
            v = (PA ? rq[PA ? k : 0] : s.r[p]) - acc;
        }
        b0[q] = v;
    }
    __syncthreads();
    const T *lay = stack_layers<T, kSAW, kSAH, NT>(b0, b1, b2, w, sx0, sy0, n);
    T k6[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) k6[k] = w[45 + k];
    for (int q = tid; q < kSAX * kSAY; q += NT) {
        const int i = X0 + q % kSAX, j = Y0 + q / kSAX;
        if (i >= n || j >= n) continue;
        const int xx = i - sx0, yy = j - sy0;
        const T v = stack_out<T, kSAW>(b0, k6, lay[yy * kSAW + xx], xx, yy);
        const T enew = pb[(yy + 1) * kSPW + xx + 1] + v;
        const int64_t p = (int64_t)j * P + i;
        if (s.u)
            s.u[p] = s.u[p] + (double)enew;
        else
            s.s[p] = enew;  // not in place: neighbouring tiles read e in their halos
    }
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

// out[0] = the mean of the centre entries of a level's stencil (fixed order: deterministic).
__global__ void __launch_bounds__(256) k_stack_mean_centre(int n, int P, int64_t plane, const double *A, double *out)
{
    __shared__ double red[4];
    double acc = 0.0;
    for (int64_t q = threadIdx.x; q < (int64_t)n * n; q += 256) acc += A[4 * plane + (q / n) * P + q % n];
    const double s = block_sum<256>(acc, red);
    if (threadIdx.x == 0) out[0] = s / ((double)n * n);
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

// ---- the levels with n <= kBottomMax in one workgroup per problem
// Every smoothing level and the coarsest are held in LDS: five vectors per
// level (r, e, s and two for the stack's intermediate layers) of (n + 2)^2
// elements with a zero border of one node, which is the zero padding of every
// layer; one thread per node (n^2 <= 961 < 1024 threads).  The V-cycle of
// these levels (Algorithm 1) runs with a workgroup barrier between steps
// instead of a launch per step; the coarsest inverse is read into LDS.  With
// prm given it also applies the solver's stopping rule to the outer residual's
// block sums, as the network smoother's bottom kernel does (k_bottom): summed
// with the first loads, applied by a thread with no top-level node, and u
// changes only if the problem goes on.
constexpr int kSBT = 1024;
constexpr int kSBVec = 5;
constexpr size_t kSBAinvBytes = ((size_t)kMaxCoarseUnknowns * kMaxCoarseUnknowns * sizeof(double) + 15) / 16 * 16;

__host__ __device__ inline int sb_vec(int n) { return (n + 2) * (n + 2); }
__device__ inline int sb_at(int n, int i, int j) { return (j + 1) * (n + 2) + i + 1; }

template <typename T>
__global__ void __launch_bounds__(kSBT) k_stack_bottom(const BottomSlot<T> *slots, SolveState *state, int nu1, int nu2,
                                                       const SolveParams *prm)
{
    __shared__ double wsum[kSBT / 64];
    __shared__ int go;
    extern __shared__ __align__(16) unsigned char sb_raw[];
    double *ainv = (double *)sb_raw;
    T *sm = (T *)(sb_raw + kSBAinvBytes);
    const BottomSlot<T> &S = slots[blockIdx.x];
    if (!state[S.prob].active) return;  // uniform over the workgroup
    const int NL = S.nlev, tid = threadIdx.x;
    int off[kMaxBottomLevels];
    int total = 0;
    for (int l = 0; l < kMaxBottomLevels; ++l) {
        off[l] = total;
        if (l < NL) total += kSBVec * sb_vec(S.lev[l].n);
    }
    const int mc = S.lev[NL - 1].n, mm = mc * mc;
    const bool check = prm != nullptr;  // uniform
    double rr0 = 0.0, rr1 = 0.0, rr2 = 0.0, rr3 = 0.0;
    if (check) {
        const int np = state[S.prob].nparts;
        int q = tid;
        for (; q + 3 * kSBT < np; q += 4 * kSBT) {
            rr0 += S.partial[q];
            rr1 += S.partial[q + kSBT];
            rr2 += S.partial[q + 2 * kSBT];
            rr3 += S.partial[q + 3 * kSBT];
        }
        for (; q < np; q += kSBT) rr0 += S.partial[q];
    }
    for (int q = tid; q < total; q += kSBT) sm[q] = (T)0;
    for (int q = tid; q < mm * mm; q += kSBT) ainv[q] = S.Ainv[q];
    if (check) {
        const double w = wave_sum((rr0 + rr1) + (rr2 + rr3));
        if ((tid & 63) == 0) wsum[tid >> 6] = w;
    }
    __syncthreads();
    if (check && tid == kSBT - 1) {  // no top-level node (n^2 <= 961)
        double rr = 0.0;
        for (int w = 0; w < kSBT / 64; ++w) rr += wsum[w];
        SolveState &st = state[S.prob];
        stopping_rule(st, rr, prm, S.prob);
        go = st.active;
    }
    {
        const int n = S.lev[0].n, P = S.lev[0].P;
        for (int q = tid; q < n * n; q += kSBT) sm[off[0] + sb_at(n, q % n, q / n)] = S.r_in[(int64_t)(q / n) * P + q % n];
    }
    __syncthreads();

    // y (+)= H x on level l (x, y: LDS vector offsets); post: the weights after the coarse correction
    auto stack = [&](int l, int X, int Y, bool acc, bool post) {
        const int n = S.lev[l].n, V = sb_vec(n), T1 = off[l] + 3 * V, T2 = off[l] + 4 * V;
        const T MG_G *w = (const T MG_G *)S.lev[l].H + (post ? kStackWeights : 0);
        const int src[5] = {X, T1, T2, T1, T2}, dst[4] = {T1, T2, T1, T2};
#pragma unroll
        for (int layer = 0; layer < 4; ++layer) {
            for (int q = tid; q < n * n; q += kSBT) {
                const int i = q % n, j = q / n;
                T v = (T)0;
#pragma unroll
                for (int t = 0; t < 9; ++t) v += w[layer * 9 + t] * sm[src[layer] + sb_at(n, i + t % 3 - 1, j + t / 3 - 1)];
                sm[dst[layer] + sb_at(n, i, j)] = v;
            }
            __syncthreads();
        }
        for (int q = tid; q < n * n; q += kSBT) {
            const int i = q % n, j = q / n;
            T v = (T)0;
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const int a = sb_at(n, i + t % 3 - 1, j + t / 3 - 1);
                v += w[36 + t] * sm[src[4] + a] + w[45 + t] * sm[X + a];
            }
            const int p = Y + sb_at(n, i, j);
            sm[p] = acc ? sm[p] + v : v;
        }
        __syncthreads();
    };
    // s = r - A e on level l
    auto residual = [&](int l) {
        const int n = S.lev[l].n, P = S.lev[l].P, V = sb_vec(n), R = off[l], E = R + V, Sv = R + 2 * V;
        const int64_t plane = S.lev[l].plane;
        for (int q = tid; q < n * n; q += kSBT) {
            const int i = q % n, j = q / n;
            T acc = (T)0;
#pragma unroll
            for (int c = 0; c < 9; ++c)
                acc += S.lev[l].A[c * plane + (int64_t)j * P + i] * sm[E + sb_at(n, i + c % 3 - 1, j + c / 3 - 1)];
            sm[Sv + sb_at(n, i, j)] = sm[R + sb_at(n, i, j)] - acc;
        }
        __syncthreads();
    };
    // r_{l+1} = R s_l (full weighting)
    auto restrict_to = [&](int l) {
        const int n = S.lev[l].n, nc = S.lev[l + 1].n, Sv = off[l] + 2 * sb_vec(n), Rc = off[l + 1];
        for (int q = tid; q < nc * nc; q += kSBT) {
            const int I = q % nc, J = q / nc, ci = 2 * I + 1, cj = 2 * J + 1;
            auto sv = [&](int di, int dj) { return sm[Sv + sb_at(n, ci + di, cj + dj)]; };
            sm[Rc + sb_at(nc, I, J)] = (T)0.0625 * (sv(-1, -1) + sv(1, -1) + sv(-1, 1) + sv(1, 1)) +
                                       (T)0.125 * (sv(0, -1) + sv(0, 1) + sv(-1, 0) + sv(1, 0)) + (T)0.25 * sv(0, 0);
        }
        __syncthreads();
    };
    // e_l += P e_{l+1} (bilinear; the coarse border is zero)
    auto prolong = [&](int l) {
        const int n = S.lev[l].n, nc = S.lev[l + 1].n, E = off[l] + sb_vec(n), Ec = off[l + 1] + sb_vec(nc);
        for (int q = tid; q < n * n; q += kSBT) {
            const int i = q % n, j = q / n;
            const int ia = (i & 1) ? (i - 1) / 2 : i / 2 - 1, ib = (i & 1) ? ia : ia + 1;
            const int ja = (j & 1) ? (j - 1) / 2 : j / 2 - 1, jb = (j & 1) ? ja : ja + 1;
            T acc = sm[Ec + sb_at(nc, ia, ja)];
            if (ib != ia) acc += sm[Ec + sb_at(nc, ib, ja)];
            if (jb != ja) {
                acc += sm[Ec + sb_at(nc, ia, jb)];
                if (ib != ia) acc += sm[Ec + sb_at(nc, ib, jb)];
            }
            const T wt = (T)(((i & 1) ? 1.0 : 0.5) * ((j & 1) ? 1.0 : 0.5));
            sm[E + sb_at(n, i, j)] += wt * acc;
        }
        __syncthreads();
    };

    for (int l = 0; l + 1 < NL; ++l) {
        const int V = sb_vec(S.lev[l].n);
        if (nu1 > 0) stack(l, off[l], off[l] + V, false, false);  // e = H r
        for (int it = 1; it < nu1; ++it) {
            residual(l);
            stack(l, off[l] + 2 * V, off[l] + V, true, false);
        }
        residual(l);
        restrict_to(l);
    }
    {  // the coarsest level: e = A^{-1} r, node (row % mc, row / mc)
        const int Rc = off[NL - 1], Ec = Rc + sb_vec(mc);
        T v = (T)0;
        if (tid < mm) {
            double acc = 0.0;
            for (int k = 0; k < mm; ++k) acc += ainv[tid * mm + k] * (double)sm[Rc + sb_at(mc, k % mc, k / mc)];
            v = (T)acc;
        }
        __syncthreads();
        if (tid < mm) sm[Ec + sb_at(mc, tid % mc, tid / mc)] = v;
        __syncthreads();
    }
    for (int l = NL - 2; l >= 0; --l) {
        const int V = sb_vec(S.lev[l].n);
        prolong(l);
        for (int q = 0; q < nu2; ++q) {
            residual(l);
            stack(l, off[l] + 2 * V, off[l] + V, true, true);
        }
    }
    if (check && !go) return;  // stopped by the rule: u keeps its value (read after the barriers above)
    {
        const int n = S.lev[0].n, P = S.lev[0].P, E = off[0] + sb_vec(n);
        for (int q = tid; q < n * n; q += kSBT) {
            const int64_t p = (int64_t)(q / n) * P + q % n;
            const T e = sm[E + sb_at(n, q % n, q / n)];
            if (S.u)
                S.u[p] = S.u[p] + (double)e;  // the fused cycle of a problem that fits here: u += e
            else
                S.e_out[p] = e;
        }
    }
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

template <typename T>
void launch_stack_descend(const CycleSlot<T> *slots, int nslots, int nc, const SolveState *state, hipStream_t st)
{
    const dim3 g((unsigned)((nc + kSDX - 1) / kSDX), (unsigned)((nc + kSDY - 1) / kSDY), (unsigned)nslots);
    if (nc <= 255)
        k_stack_descend<T, 1024><<<g, 1024, 0, st>>>(slots, state);
    else
        k_stack_descend<T, kST><<<g, kST, 0, st>>>(slots, state);
}
template <typename T>
void launch_stack_ascend(const CycleSlot<T> *slots, int nslots, int n, const SolveState *state, hipStream_t st)
{
    // the stencil in registers costs occupancy: only where the grid is too small to hide latency anyway.
    // Above n = 511, 512 threads (two passes over the 76 x 28 e' region instead of nine): at n = 1023
    // 19.8 us per launch against 24.5 with 256 threads, 23.3 with 768, 22.4 with the stencil in registers
    if (n > 511)
        k_stack_ascend<T, false, 512><<<tile_grid(n, nslots), 512, 0, st>>>(slots, state);
    else if (sizeof(T) == 4)
        k_stack_ascend<T, true, 1024><<<tile_grid(n, nslots), 1024, 0, st>>>(slots, state);
    else
        k_stack_ascend<T, false, 1024><<<tile_grid(n, nslots), 1024, 0, st>>>(slots, state);
}
template void launch_stack_descend<float>(const CycleSlot<float> *, int, int, const SolveState *, hipStream_t);
template void launch_stack_descend<double>(const CycleSlot<double> *, int, int, const SolveState *, hipStream_t);
template void launch_stack_ascend<float>(const CycleSlot<float> *, int, int, const SolveState *, hipStream_t);
template void launch_stack_ascend<double>(const CycleSlot<double> *, int, int, const SolveState *, hipStream_t);

template <typename T>
size_t stack_bottom_smem_bytes(int top_n)
{
    size_t v = 0;
    for (int m = top_n, l = 0; l < kMaxBottomLevels; ++l, m = m > 1 ? (m - 1) / 2 : 1) v += kSBVec * sb_vec(m);
    return kSBAinvBytes + v * sizeof(T);
}

template <typename T>
void prepare_stack_bottom()
{
    // allow more than 64 KiB of dynamic LDS
    (void)hipFuncSetAttribute((const void *)k_stack_bottom<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)stack_bottom_smem_bytes<T>(kBottomMax));
}

template <typename T>
void launch_stack_bottom(const BottomSlot<T> *slots, int nslots, int top_n, int nu1, int nu2, SolveState *state,
                         const SolveParams *prm, hipStream_t st)
{
    k_stack_bottom<T><<<nslots, kSBT, stack_bottom_smem_bytes<T>(top_n), st>>>(slots, state, nu1, nu2, prm);
}
template void prepare_stack_bottom<float>();
template void prepare_stack_bottom<double>();
template void launch_stack_bottom<float>(const BottomSlot<float> *, int, int, int, int, SolveState *,
                                         const SolveParams *, hipStream_t);
template void launch_stack_bottom<double>(const BottomSlot<double> *, int, int, int, int, SolveState *,
                                          const SolveParams *, hipStream_t);

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

void launch_stack_mean_centre(int n, int P, int64_t plane, const double *A, double *out, hipStream_t st)
{
    k_stack_mean_centre<<<1, 256, 0, st>>>(n, P, plane, A, out);
}

void launch_stack_adam(double *w, double *m, double *v, const double *g, int t, double lr, double b1, double b2,
                       double eps, hipStream_t st)
{
    k_stack_adam<<<1, 64, 0, st>>>(w, m, v, g, t, lr, b1, b2, eps);
}

}  // namespace mg
