// BF16 training path of the stencil-to-smoother network on the matrix cores.
// Activations are stored channel-last in BF16 ([pixel][channel], 16 channels
// for the network input, 32 for hidden layers and gradients); the last
// layer's output is kept in FP32.  Every convolution is an implicit GEMM on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation:
//   forward       out[p][co] = sum_{tap,ci} in[p + tap][ci] W[co][ci][tap]  (M = pixels)
//   data gradient dX[q][ci]  = sum_{tap,co} dY[q - tap][co] W[co][ci][tap] (the same GEMM with
//                 the transposed, flipped weights; masked by the ReLU of the forward pass)
//   weight grad.  dW[tap][co][ci] = sum_p dY[p][co] X[p + tap][ci]         (M = co, N = ci, K = pixels)
// Workgroups take 16 x 16 tiles of one problem; weight gradients are written
// per tile and reduced in a fixed order (deterministic).
//
// MFMA operand layout (16x16x32, wave of 64): lane l supplies
// A[m = l % 16][k = 8 (l / 16) + e], B[k = 8 (l / 16) + e][n = l % 16],
// and receives C[m = 4 (l / 16) + i][n = l % 16].
#include "common.hpp"
#include "train.hpp"

namespace mg {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kT = 256;
constexpr int kTile = 16;
constexpr int kHalo = kTile + 2;
constexpr int ceil_div(int a, int b) { return (a + b - 1) / b; }

__device__ inline bool in_grid(int n, int i, int j) { return i >= 0 && i < n && j >= 0 && j < n; }

// Tensor selector of a TrainProbB.
__device__ inline bf16_t MG_G *bsel(const TrainProbB &P, int which)
{
    switch (which) {
    case kTbX0: return P.x0;
    case kTbAct0: return P.act;
    case kTbAct1: return P.act + P.plane * 32;
    case kTbAct2: return P.act + P.plane * 64;
    case kTbDA: return P.dA;
    default: return P.dB;
    }
}

// One convolution layer on a 16 x 16 tile.  EPI: 0 forward hidden layer
// (bias, ReLU, zero off the grid, BF16 out); 1 forward last layer (bias,
// FP32 out to y); 2 data gradient (mask by the forward activation `mask`).
template <int CSIN, int STEPS, bool FIRST, int EPI>
__global__ void __launch_bounds__(kT) k_trb_conv(const TrainProbB *probs, const bf16_t *wpack, const float *bias,
                                                 int in_sel, int out_sel, int mask_sel)
{
    // pixel stride CSIN + 8 bf16 (12 or 20 dwords): the 16 pixels of one lane group's ds_read_b128
    // start in distinct groups of four banks (a stride of CSIN puts two or four lanes on one group)
    constexpr int LD = CSIN + 8;
    __shared__ __align__(16) bf16_t tin[kHalo * kHalo * LD];
    const TrainProbB &P = probs[blockIdx.z];
    const int n = P.n;
    const int X0 = blockIdx.x * kTile, Y0 = blockIdx.y * kTile;
    if (X0 >= n || Y0 >= n) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4;
    const bf16_t MG_G *in = bsel(P, in_sel);
    // input tile with a halo of one, zero off the grid: 16-byte chunks of 8 channels
    constexpr int CH = CSIN / 8;
    for (int q = tid; q < kHalo * kHalo * CH; q += kT) {
        const int pix = q / CH, c8 = q % CH;
        const int gi = X0 - 1 + pix % kHalo, gj = Y0 - 1 + pix / kHalo;
        const bool ok = in_grid(n, gi, gj);
        const int64_t p = ok ? (int64_t)gj * n + gi : 0;
        u32x4 v = *(const u32x4 MG_G *)(in + p * CSIN + c8 * 8);
        if (!ok) v = u32x4{0u, 0u, 0u, 0u};
        *(u32x4 *)(tin + pix * LD + c8 * 8) = v;
    }
    bf16x8 bw[STEPS][2];
    const bf16_t MG_G *wp = (const bf16_t MG_G *)wpack;
#pragma unroll
    for (int s = 0; s < STEPS; ++s)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) bw[s][nb] = *(const bf16x8 MG_G *)(wp + ((s * 2 + nb) * 64 + lane) * 8);
    const float b0 = bias ? bias[lane & 15] : 0.f, b1 = bias ? bias[16 + (lane & 15)] : 0.f;
    __syncthreads();
    for (int mb = wave; mb < kTile * kTile / 16; mb += kT / 64) {
        const int pa = mb * 16 + (lane & 15);
        const int oy = pa / kTile, ox = pa % kTile;
        f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
        // data gradient: the forward activations that mask it, loaded before the products so that
        // their latency overlaps them (clamped address off the grid, unused there)
        bf16_t mk0[4], mk1[4];
        if (EPI == 2) {
            const bf16_t MG_G *m = bsel(P, mask_sel);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int pix = mb * 16 + 4 * g + i;
                const int gi = X0 + pix % kTile, gj = Y0 + pix / kTile;
                const int64_t p = (gi < n && gj < n) ? (int64_t)gj * n + gi : 0;
                mk0[i] = m[p * 32 + (lane & 15)];
                mk1[i] = m[p * 32 + 16 + (lane & 15)];
            }
        }
#pragma unroll
        for (int s = 0; s < STEPS; ++s) {
            int tap, cg;
            if (FIRST) {
                tap = 2 * s + (g >> 1);
                cg = g & 1;
            } else {
                tap = s;
                cg = g;
            }
            bf16x8 a;
            if (FIRST && tap > 8) {
                a = bf16x8{};
            } else {
                const int ky = tap / 3, kx = tap - 3 * (tap / 3);
                a = *(const bf16x8 *)(tin + ((oy + ky) * kHalo + ox + kx) * LD + cg * 8);
            }
            acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[s][0], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[s][1], acc1, 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int pix = mb * 16 + 4 * g + i;
            const int gi = X0 + pix % kTile, gj = Y0 + pix / kTile;
            if (gi >= n || gj >= n) continue;
            const int64_t p = (int64_t)gj * n + gi;
            const int c0 = lane & 15, c1 = 16 + (lane & 15);
            float v0 = acc0[i] + b0, v1 = acc1[i] + b1;
            if (EPI == 0) {
                bf16_t MG_G *out = bsel(P, out_sel);
                out[p * 32 + c0] = f32_to_bf16(v0 > 0.f ? v0 : 0.f);
                out[p * 32 + c1] = f32_to_bf16(v1 > 0.f ? v1 : 0.f);
            } else if (EPI == 1) {
                P.y[p * 32 + c0] = v0;
                P.y[p * 32 + c1] = v1;
            } else {
                bf16_t MG_G *out = bsel(P, out_sel);
                out[p * 32 + c0] = f32_to_bf16(bf16_to_f32(mk0[i]) > 0.f ? v0 : 0.f);
                out[p * 32 + c1] = f32_to_bf16(bf16_to_f32(mk1[i]) > 0.f ? v1 : 0.f);
            }
        }
    }
}

// Weight and bias gradient of one layer on a group of kTileGroup consecutive
// 16 x 16 tiles of one problem (row-major tile order):
//   part[tap][co][ci] = sum_{p in group} dY[p][co] X[p + tap][ci],  part_b[co] = sum_p dY[p][co],
// accumulated tile after tile in the MFMA accumulators, so that a group writes
// one part (a quarter of the traffic of one part per tile).  Per tile, dY and X
// are staged channel-major in LDS so that a lane's eight K values (eight
// consecutive pixels of one channel) are contiguous.
// 8 waves per workgroup: the LDS of the shifted input copies allows two workgroups per CU
constexpr int kTW = 512;

template <int CIN>
__global__ void __launch_bounds__(kTW) k_trb_wgrad(const TrainProbB *probs, int dy_sel, int x_sel, int cout,
                                                  float *part)
{
    // rows padded by 8 bf16 (132 dwords): the 16 channel rows one lane group reads with ds_read_b128
    // start in distinct groups of four banks (256 would put them all on one)
    __shared__ __align__(16) bf16_t dyT[32][kTile * kTile + 8];
    // the input tile with its halo, once per horizontal tap offset kx: xS[kx][ci][row][px] = x(row, px + kx),
    // so that a lane's eight consecutive pixels of a tap are one aligned 16-byte read; channel stride
    // 18 * 16 + 8 (148 dwords) keeps the sixteen channels of a lane group on distinct bank groups
    constexpr int XS = kHalo * kTile + 8;
    __shared__ __align__(16) bf16_t xS[3][CIN][XS];
    __shared__ float bred[16][32];
    const TrainProbB &P = probs[blockIdx.z];
    const int n = P.n;
    const int tiles = (n + kTile - 1) / kTile, ntile = tiles * tiles;
    const int t0 = blockIdx.x * kTileGroup, t1 = min(ntile, t0 + kTileGroup);
    if (t0 >= ntile) return;
    float *out = part + ((int64_t)P.part0 + blockIdx.x) * (9 * 32 * 32 + 32);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4;
    const bf16_t MG_G *dy = bsel(P, dy_sel);
    const bf16_t MG_G *x = bsel(P, x_sel);
    // (tap, ci-block) jobs of one co-block per wave (waves 2q and 2q + 1: co-blocks 0 and 1, jobs
    // q, q + 4, ..), so that a wave's A fragment (dY of its co-block) serves all its jobs per K step
    constexpr int NB = CIN / 16, NJB = 9 * NB, JPW = (NJB + 3) / 4;
    const int wmb = wave & 1, wq = wave >> 1;
    f32x4 acc[JPW];
#pragma unroll
    for (int jj = 0; jj < JPW; ++jj) acc[jj] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bacc = 0.f;
    // Staging: a work item loads one 8-channel chunk of 8 consecutive pixels (eight 16-byte loads),
    // transposes the 8 x 8 block in registers and writes 8 channel rows of 8 pixels (16 bytes each).
    constexpr int CH = CIN / 8;
    constexpr int NDY = kTile * kTile / 8 * 4, NXS = 3 * kHalo * 2 * CH;
    // rows[c] = the 8 values of channel c of the 8 chunks v[0..7] (pixel e in position e)
    auto transpose8 = [](const u32x4 (&v)[8], u32x4 (&rows)[8]) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            uint32_t w[4];
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const uint32_t a = v[2 * h][c / 2], b = v[2 * h + 1][c / 2];
                w[h] = (c & 1) ? ((a >> 16) | (b & 0xffff0000u)) : ((a & 0xffffu) | (b << 16));
            }
            rows[c] = u32x4{w[0], w[1], w[2], w[3]};
        }
    };
    for (int t = t0; t < t1; ++t) {
        // (the barrier at the end of the previous tile: its products are done with the LDS)
        const int X0 = (t % tiles) * kTile, Y0 = (t / tiles) * kTile;
        for (int item = tid; item < NDY + NXS; item += kTW) {
          if (item < NDY) {
            const int pb = item / 4, c8 = item % 4;  // pixels 8 pb .. 8 pb + 7 of the tile (one half row)
            u32x4 v[8], rows[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int pix = pb * 8 + e;
                const int gi = X0 + pix % kTile, gj = Y0 + pix / kTile;
                const bool ok = in_grid(n, gi, gj);
                const int64_t p = ok ? (int64_t)gj * n + gi : 0;
                const u32x4 ld = *(const u32x4 MG_G *)(dy + p * 32 + c8 * 8);
                v[e] = ok ? ld : u32x4{0u, 0u, 0u, 0u};
            }
            transpose8(v, rows);
#pragma unroll
            for (int c = 0; c < 8; ++c) *(u32x4 *)&dyT[c8 * 8 + c][pb * 8] = rows[c];
          } else {
            // xS[kx][ci][row][px0 .. px0 + 7] = x(row, px0 + kx ..) in halo coordinates
            const int w = item - NDY;
            const int c8 = w % CH, seg = (w / CH) % 2, row = (w / (2 * CH)) % kHalo, kx = w / (2 * CH * kHalo);
            const int px0 = seg * 8;
            u32x4 v[8], rows[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int gi = X0 - 1 + px0 + kx + e, gj = Y0 - 1 + row;
                const bool ok = in_grid(n, gi, gj);
                const int64_t p = ok ? (int64_t)gj * n + gi : 0;
                const u32x4 ld = *(const u32x4 MG_G *)(x + p * CIN + c8 * 8);
                v[e] = ok ? ld : u32x4{0u, 0u, 0u, 0u};
            }
            transpose8(v, rows);
#pragma unroll
            for (int c = 0; c < 8; ++c) *(u32x4 *)&xS[kx][c8 * 8 + c][row * kTile + px0] = rows[c];
          }
        }
        __syncthreads();
        // bias gradient: 16 partial sums of 16 pixels per channel (all threads), combined in order by
        // the first 32 threads after the tile's products
        {
            const int c = tid & 31, part16 = tid >> 5;
            float sacc = 0.f;
#pragma unroll
            for (int p = 0; p < 16; ++p) sacc += bf16_to_f32(dyT[c][part16 * 16 + p]);
            bred[part16][c] = sacc;
        }
        static_assert(kTW == 8 * 64, "eight waves: two co-blocks x four job sets");
        const int co = wmb * 16 + (lane & 15);
#pragma unroll 2
        for (int ks = 0; ks < kTile * kTile / 32; ++ks) {
            const int k0 = ks * 32 + 8 * g;  // eight consecutive pixels of one tile row
            const int py = k0 / kTile, px = k0 % kTile;
            const bf16x8 a = *(const bf16x8 *)&dyT[co][k0];
#pragma unroll
            for (int jj = 0; jj < JPW; ++jj) {
                const int q = wq + 4 * jj;
                if (q >= NJB) break;
                const int tap = q / NB, nb = q % NB;
                const int ky = tap / 3, kx = tap % 3;
                const int ci = nb * 16 + (lane & 15);
                const bf16x8 b = *(const bf16x8 *)&xS[kx][ci][(py + ky) * kTile + px];
                acc[jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[jj], 0, 0, 0);
            }
        }
        __syncthreads();  // bred complete
        if (tid < 32) {
            float sacc = 0.f;
            for (int q = 0; q < 16; ++q) sacc += bred[q][tid];
            bacc += sacc;
        }
    }
    if (tid < 32) out[9 * 32 * 32 + tid] = tid < cout ? bacc : 0.f;
    static_assert(kTW == 16 * 32, "one thread per (16-pixel part, channel) of the bias gradient");
#pragma unroll
    for (int jj = 0; jj < JPW; ++jj) {
        const int q = wq + 4 * jj;
        if (q >= NJB) break;
        const int tap = q / NB, nb = q % NB;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int co_i = wmb * 16 + 4 * g + i;
            out[(tap * 32 + co_i) * 32 + nb * 16 + (lane & 15)] = acc[jj][i];
        }
    }
}

// x0 = A / a_C, channel-last BF16 with 16 channels (9 used).
__global__ void __launch_bounds__(kT) k_trb_input(const TrainProbB *probs)
{
    const TrainProbB &P = probs[blockIdx.z];
    const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (p >= P.plane) return;
    const double ac = P.A[kCentre * P.plane + p];
    for (int c = 0; c < 16; ++c) P.x0[p * 16 + c] = f32_to_bf16(c < 9 ? (float)(P.A[c * P.plane + p] / ac) : 0.f);
}

// Av_j = A v_j for every vector of a problem, one thread per pixel: the nine
// stencil entries are read once for all J vectors.  grid.z = problem.
__global__ void __launch_bounds__(kT) k_trb_av(const TrainProbB *probs, int J)
{
    const TrainProbB &P = probs[blockIdx.z];
    const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (p >= P.plane) return;
    const int n = P.n, i = (int)(p % n), j = (int)(p / n);
    float a[9];
    int64_t off[9];
    bool ok[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) {
        const int ii = i + c % 3 - 1, jj = j + c / 3 - 1;
        ok[c] = in_grid(n, ii, jj);
        off[c] = ok[c] ? (int64_t)jj * n + ii : p;
        a[c] = (float)P.A[c * P.plane + p];
    }
    for (int jv = 0; jv < J; ++jv) {
        const float MG_G *v = P.V + (int64_t)jv * P.plane;
        float acc = 0.0f;
#pragma unroll
        for (int c = 0; c < 9; ++c) {
            const float xv = v[off[c]];
            acc += a[c] * (ok[c] ? xv : 0.f);
        }
        P.Av[(int64_t)jv * P.plane + p] = acc;
    }
}

// The rows of A v_j that a block of kT consecutive pixels reaches with the 5 x 5 smoother (two
// above its first row, two below its last) are staged in LDS, double-buffered: while vector j is
// computed from one buffer, the rows of vector j + 1 are loaded into registers and then stored to
// the other, so that one barrier per vector separates them and the loads overlap the arithmetic.
constexpr int kResRows = 1792;  // >= max over 3 <= n <= 255 of (255 / n + 6) n
constexpr int kRowRegs = kResRows / kT;  // staged values per thread
static_assert(kRowRegs * kT == kResRows, "whole rounds of staging");

struct BlockRows {
    int r0, nrow;
};

__device__ inline BlockRows block_rows(int64_t plane, int n)
{
    const int64_t p0 = (int64_t)blockIdx.x * kT, p1 = min(p0 + kT, plane) - 1;
    const int r0 = max(0, (int)(p0 / n) - 2), r1 = min(n - 1, (int)(p1 / n) + 2);
    return {r0, (r1 - r0 + 1) * n};  // nrow <= (255 / n + 6) n <= 1785 for 3 <= n <= 255
}

__device__ inline void load_rows(const TrainProbB &P, const BlockRows &br, int jv, float (&r)[kRowRegs])
{
    const float MG_G *Av = P.Av + (int64_t)jv * P.plane + (int64_t)br.r0 * P.n;
#pragma unroll
    for (int k = 0; k < kRowRegs; ++k) {
        const int t = threadIdx.x + k * kT;
        r[k] = t < br.nrow ? Av[t] : 0.f;
    }
}

__device__ inline void store_rows(const BlockRows &br, const float (&r)[kRowRegs], float *buf)
{
#pragma unroll
    for (int k = 0; k < kRowRegs; ++k) {
        const int t = threadIdx.x + k * kT;
        if (t < br.nrow) buf[t] = r[k];
    }
}

// g_j = v_j - H A v_j for every vector j of a problem, one thread per pixel:
// the pixel's 25 smoother taps are read once for all J vectors.  Per block and
// vector, the sum of g_j^2 (FP64, waves then the block in a fixed order) goes
// to part[problem][block][j].  grid = (pixel blocks, 1, problems).
constexpr int kJChunk = 64;
__global__ void __launch_bounds__(kT) k_trb_residual(const TrainProbB *probs, int J, float omega, double *part,
                                                     int nblk)
{
    __shared__ double red[kT / 64][kJChunk];
    __shared__ float sav[2][kResRows];
    const TrainProbB &P = probs[blockIdx.z];
    const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
    const bool live = p < P.plane;
    const int n = P.n;
    const int64_t pc = live ? p : 0;
    const int i = (int)(pc % n), j = (int)(pc / n);
    const BlockRows br = block_rows(P.plane, n);
    float rows[kRowRegs];
    load_rows(P, br, 0, rows);
    float w[25];
#pragma unroll
    for (int k = 0; k < 25; ++k) w[k] = P.y[pc * 32 + k] + (k == 12 ? omega : 0.0f);
    const float inv_ac = 1.0f / (float)P.A[kCentre * P.plane + pc];
    int off[25];
    bool ok[25];
#pragma unroll
    for (int k = 0; k < 25; ++k) {
        const int ii = i + k % 5 - 2, jj = j + k / 5 - 2;
        ok[k] = live && in_grid(n, ii, jj);
        off[k] = ok[k] ? (jj - br.r0) * n + ii : 0;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double *out = part + ((int64_t)P.index * nblk + blockIdx.x) * J;
    store_rows(br, rows, sav[0]);
    float vnext = P.V[pc];
    __syncthreads();
    for (int j0 = 0; j0 < J; j0 += kJChunk) {
        const int jn = min(kJChunk, J - j0);
        for (int q = 0; q < jn; ++q) {
            const int jv = j0 + q;
            const float vj = vnext;
            if (jv + 1 < J) {  // the next vector's rows and value, in flight during this one
                load_rows(P, br, jv + 1, rows);
                vnext = P.V[(int64_t)(jv + 1) * P.plane + pc];
            }
            const float *buf = sav[jv & 1];
            float y = 0.0f;
#pragma unroll
            for (int k = 0; k < 25; ++k) {
                const float xv = buf[off[k]];
                y += w[k] * (ok[k] ? xv : 0.f);
            }
            const float gv = vj - y * inv_ac;
            if (live) P.g[(int64_t)jv * P.plane + p] = gv;
            const double s = wave_sum(live ? (double)gv * gv : 0.0);
            if (lane == 0) red[wave][q] = s;
            if (jv + 1 < J) store_rows(br, rows, sav[(jv + 1) & 1]);
            __syncthreads();  // the next vector's rows are in LDS; this vector's buffer is free
        }
        if ((int)threadIdx.x < jn) {
            double s = 0.0;
            for (int w2 = 0; w2 < kT / 64; ++w2) s += red[w2][threadIdx.x];
            out[j0 + threadIdx.x] = s;
        }
        __syncthreads();  // red is reused by the next chunk
    }
}

// ||g_j|| from the block sums, in block order; one thread per vector.
__global__ void k_trb_norms(const TrainProbB *probs, int J, const double *part, int nblk, float *loss_part)
{
    const TrainProbB &P = probs[blockIdx.x];
    const int nb = (int)((P.plane + kT - 1) / kT);
    for (int jv = threadIdx.x; jv < J; jv += blockDim.x) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += part[((int64_t)P.index * nblk + b) * J + jv];
        const float gn = (float)sqrt(s);
        P.gnorm[jv] = gn;
        loss_part[P.index * J + jv] = gn;
    }
}

// dL/dy_p[k] = -(1/(B J)) sum_j (g_j(p)/||g_j||) Av_j(p + k)/a_C(p) -> dA (channel-last BF16, 32
// channels), the rows of A v_j staged in LDS as for the residual.
__global__ void __launch_bounds__(kT) k_trb_dout(const TrainProbB *probs, int J, float scale)
{
    __shared__ float sav[2][kResRows];
    const TrainProbB &P = probs[blockIdx.z];
    const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
    const bool live = p < P.plane;
    const int n = P.n;
    const int64_t pc = live ? p : 0;
    const int i = (int)(pc % n), j = (int)(pc / n);
    const BlockRows br = block_rows(P.plane, n);
    float rows[kRowRegs];
    load_rows(P, br, 0, rows);
    const float inv_ac = 1.0f / (float)P.A[kCentre * P.plane + pc];
    int off[25];
    bool ok[25];
#pragma unroll
    for (int k = 0; k < 25; ++k) {
        const int ii = i + k % 5 - 2, jj = j + k / 5 - 2;
        ok[k] = live && in_grid(n, ii, jj);
        off[k] = ok[k] ? (jj - br.r0) * n + ii : 0;
    }
    float acc[25];
#pragma unroll
    for (int k = 0; k < 25; ++k) acc[k] = 0.0f;
    store_rows(br, rows, sav[0]);
    float gnext = P.g[pc];
    __syncthreads();
    for (int jv = 0; jv < J; ++jv) {
        const float gj = gnext;
        if (jv + 1 < J) {  // the next vector's rows and residual, in flight during this one
            load_rows(P, br, jv + 1, rows);
            gnext = P.g[(int64_t)(jv + 1) * P.plane + pc];
        }
        const float gn = P.gnorm[jv];
        const float c = gn > 0.f ? -scale * gj / gn * inv_ac : 0.f;
        const float *buf = sav[jv & 1];
#pragma unroll
        for (int k = 0; k < 25; ++k) {
            const float xv = buf[off[k]];
            acc[k] += c * (ok[k] ? xv : 0.f);
        }
        if (jv + 1 < J) store_rows(br, rows, sav[(jv + 1) & 1]);
        __syncthreads();  // the next vector's rows are in LDS; this vector's buffer is free
    }
    if (!live) return;
    // 32 channels (25 used) in four 16-byte stores
    u32x4 *o = (u32x4 *)(P.dA + p * 32);
#pragma unroll
    for (int c8 = 0; c8 < 4; ++c8) {
        uint32_t w4[4];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const int k0 = c8 * 8 + 2 * h, k1 = k0 + 1;
            const uint32_t lo = f32_to_bf16(k0 < 25 ? acc[k0 < 25 ? k0 : 0] : 0.f);
            const uint32_t hi = f32_to_bf16(k1 < 25 ? acc[k1 < 25 ? k1 : 0] : 0.f);
            w4[h] = lo | (hi << 16);
        }
        o[c8] = u32x4{w4[0], w4[1], w4[2], w4[3]};
    }
}

// grad[flat] = sum over tiles of the per-tile parts, in two deterministic
// stages.  Stage 1: block (column block, slice) sums the tiles of its slice
// for 64 consecutive columns (4 row groups, interleaved tiles, combined in
// order in LDS) into part2[slice][column].  Stage 2: one thread per parameter
// sums the slices in order and scatters to the flat layout.
constexpr int kPartCols = 9 * 32 * 32 + 32;
constexpr int kReduceSlices = 32;
__global__ void __launch_bounds__(kT) k_trb_reduce_slices(const float *part, int ntiles, float *part2)
{
    __shared__ float red[4][64];
    const int c = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const int col = blockIdx.x * 64 + c;
    const int per = (ntiles + kReduceSlices - 1) / kReduceSlices;
    const int t0 = blockIdx.y * per, t1 = min(ntiles, t0 + per);
    float s = 0.f;
    if (col < kPartCols)
        for (int t = t0 + grp; t < t1; t += 4) s += part[(int64_t)t * kPartCols + col];
    red[grp][c] = s;
    __syncthreads();
    if (grp == 0 && col < kPartCols)
        part2[(int64_t)blockIdx.y * kPartCols + col] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
}

__global__ void __launch_bounds__(kT) k_trb_reduce(const float *part2, int cin, int cout, int64_t woff,
                                                   int64_t boff, float *grad)
{
    const int q = blockIdx.x * kT + threadIdx.x;
    const int nw = cout * cin * 9;
    if (q >= nw + cout) return;
    int64_t src, dst;
    if (q < nw) {
        const int co = q / (cin * 9), ci = (q / 9) % cin, tap = q % 9;
        src = (tap * 32 + co) * 32 + ci;
        dst = woff + q;
    } else {
        src = 9 * 32 * 32 + (q - nw);
        dst = boff + (q - nw);
    }
    float s = 0.f;
    for (int t = 0; t < kReduceSlices; ++t) s += part2[(int64_t)t * kPartCols + src];
    grad[dst] = s;
}

// Per-lane B fragments: forward weights of layer l (mode 0) or the transposed,
// flipped weights for the data gradient of layer l (mode 1: B[k = co][n = ci] =
// W[co][ci][8 - tap]).  Layout [step][n-block][lane][8].
// One launch packs every layer: grid.y = job, 0..3 the forward fragments of layers 0..3, 4..6 the
// transposed ones of layers 1..3, 7..10 the padded biases of layers 0..3.
__global__ void k_trb_pack_all(const float *params, TrbPackJobs jobs)
{
    const int job = blockIdx.y;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (job >= 7) {
        const TrainLayer &L = jobs.layer[job - 7];
        if (idx < 32) jobs.bias[job - 7][idx] = idx < L.cout ? params[L.boff + idx] : 0.f;
        return;
    }
    const int mode = job < 4 ? 0 : 1, layer = job < 4 ? job : job - 3;
    const bool first = mode == 0 && layer == 0;
    const int steps = first ? 5 : 9;
    if (idx >= steps * 2 * 64 * 8) return;
    const TrainLayer &L = jobs.layer[layer];
    const int cin = L.cin, cout = L.cout;
    const int e = idx & 7, lane = (idx >> 3) & 63, nb = (idx >> 9) & 1, s = idx >> 10;
    const int g = lane >> 4, col = nb * 16 + (lane & 15);
    float v = 0.f;
    if (mode == 0) {
        int tap, ci;
        if (first) {
            tap = 2 * s + (g >> 1);
            ci = 8 * (g & 1) + e;
        } else {
            tap = s;
            ci = 8 * g + e;
        }
        const int co = col;
        if (tap < 9 && ci < cin && co < cout) v = params[L.woff + ((int64_t)co * cin + ci) * 9 + tap];
    } else {
        const int tap = s, co = 8 * g + e, ci = col;
        if (co < cout && ci < cin) v = params[L.woff + ((int64_t)co * cin + ci) * 9 + (8 - tap)];
    }
    (mode == 0 ? jobs.fwd[layer] : jobs.bwd[layer])[idx] = f32_to_bf16(v);
}

inline unsigned blocks_for(int64_t count) { return (unsigned)((count + kT - 1) / kT); }

}  // namespace

void launch_trb_pack_all(const float *params, const TrbPackJobs &jobs, hipStream_t st)
{
    k_trb_pack_all<<<dim3(blocks_for(9 * 2 * 64 * 8), 11), kT, 0, st>>>(params, jobs);
}

void launch_trb_input(const TrainProbB *probs, int nb, int n, hipStream_t st)
{
    k_trb_input<<<dim3(blocks_for((int64_t)n * n), 1, nb), kT, 0, st>>>(probs);
}

void launch_trb_conv_fwd(const TrainProbB *probs, int nb, int n, int layer, const bf16_t *wpack, const float *bias,
                         hipStream_t st)
{
    const int t = (n + kTile - 1) / kTile;
    const dim3 g(t, t, nb);
    if (layer == 0)
        k_trb_conv<16, 5, true, 0><<<g, kT, 0, st>>>(probs, wpack, bias, kTbX0, kTbAct0, 0);
    else if (layer < 3)
        k_trb_conv<32, 9, false, 0><<<g, kT, 0, st>>>(probs, wpack, bias, kTbAct0 + layer - 1, kTbAct0 + layer, 0);
    else
        k_trb_conv<32, 9, false, 1><<<g, kT, 0, st>>>(probs, wpack, bias, kTbAct2, 0, 0);
}

void launch_trb_conv_bwd_data(const TrainProbB *probs, int nb, int n, int layer, const bf16_t *wpack_t,
                              hipStream_t st)
{
    // the gradient of layer `layer`'s output is in dA for layers 3 and 1, dB for layer 2
    const int t = (n + kTile - 1) / kTile;
    const dim3 g(t, t, nb);
    const int in_sel = (layer & 1) ? kTbDA : kTbDB, out_sel = (layer & 1) ? kTbDB : kTbDA;
    k_trb_conv<32, 9, false, 2><<<g, kT, 0, st>>>(probs, wpack_t, nullptr, in_sel, out_sel, kTbAct0 + layer - 1);
}

void launch_trb_wgrad(const TrainProbB *probs, int nb, int n, int layer, int cout, float *part, hipStream_t st)
{
    const dim3 g(trb_tile_groups(n), 1, nb);
    const int dy_sel = (layer & 1) ? kTbDA : kTbDB;
    if (layer == 0)
        k_trb_wgrad<16><<<g, kTW, 0, st>>>(probs, dy_sel, kTbX0, cout, part);
    else
        k_trb_wgrad<32><<<g, kTW, 0, st>>>(probs, dy_sel, kTbAct0 + layer - 1, cout, part);
}

void launch_trb_reduce(const float *part, int ntiles, int cin, int cout, int64_t woff, int64_t boff, float *grad,
                       float *part2, hipStream_t st)
{
    k_trb_reduce_slices<<<dim3((kPartCols + 63) / 64, kReduceSlices), kT, 0, st>>>(part, ntiles, part2);
    k_trb_reduce<<<blocks_for(cout * cin * 9 + cout), kT, 0, st>>>(part2, cin, cout, woff, boff, grad);
}

size_t trb_reduce_scratch_bytes() { return sizeof(float) * (size_t)kReduceSlices * kPartCols; }

void launch_trb_av(const TrainProbB *probs, int nb, int n, int J, hipStream_t st)
{
    k_trb_av<<<dim3(blocks_for((int64_t)n * n), 1, nb), kT, 0, st>>>(probs, J);
}

void launch_trb_residual_norm(const TrainProbB *probs, int nb, int n, int J, float omega, float *loss_part,
                              double *part, int nblk, hipStream_t st)
{
    k_trb_residual<<<dim3(blocks_for((int64_t)n * n), 1, nb), kT, 0, st>>>(probs, J, omega, part, nblk);
    k_trb_norms<<<nb, 64, 0, st>>>(probs, J, part, nblk, loss_part);
}

int trb_residual_blocks(int nmax) { return (int)blocks_for((int64_t)nmax * nmax); }

void launch_trb_dout(const TrainProbB *probs, int nb, int n, int J, float scale, hipStream_t st)
{
    k_trb_dout<<<dim3(blocks_for((int64_t)n * n), 1, nb), kT, 0, st>>>(probs, J, scale);
}

}  // namespace mg
