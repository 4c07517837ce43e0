// Smoother inference on the matrix cores (paper section 4.2: the network maps
// the field of operator stencils to per-point smoothing kernels), all four
// layers of 3x3 convolutions (9 -> 32 -> 32 -> 32 -> 25) in one kernel.
//
// Each workgroup produces a kTO x kTO tile of smoother stencils; one launch
// covers every level of every problem (a table of levels, tiles numbered
// level after level).  It reads
// the stencil field on the tile plus a halo of four nodes (one per layer),
// forms the network input x0 = A / a_C, and runs the layers on shrinking
// regions (tile + 6, + 4, + 2, + 0), keeping the activations in LDS in BF16,
// channel-last (pixel-major, 32 channels per pixel).  Each layer is an
// implicit GEMM: M = pixels, N = output channels, K = (tap, input channel),
// on v_mfma_f32_16x16x32_bf16 with FP32 accumulation.  The first layer's nine
// input channels are padded to sixteen, so one K step of 32 covers two taps.
// Activations at nodes outside the grid are set to zero after every layer:
// this is the per-layer zero padding of "same" convolutions.  The last layer
// writes H = (omega*delta_0 + y) / a_C in BF16 (y = 0 on rows whose
// off-centre entries do not sum to a negative value).
//
// MFMA operand layout used (16x16x32, wave of 64): lane l supplies
// A[m = l % 16][k = 8 (l / 16) + e] and B[k = 8 (l / 16) + e][n = l % 16],
// e = 0..7, and receives C[m = 4 (l / 16) + i][n = l % 16], i = 0..3.
#include "common.hpp"
#include "launch.hpp"

namespace mg {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kTO = 16;                       // output tile side
constexpr int kT = 512;                       // 8 waves: with two workgroups per CU (LDS-bound), four waves per SIMD
constexpr int kR0 = kTO + 8, kR1 = kTO + 6, kR2 = kTO + 4, kR3 = kTO + 2;
// channel strides (bf16) of the input and hidden buffers: 16 and 32 channels padded to 24 and 40, so
// that the 16 pixels a ds_read_b128 of one lane group reads start in distinct groups of four banks
// (strides of 12 and 20 dwords; 8 and 16 dwords put four lanes on one bank group)
constexpr int kCS0 = 24, kCS = 40;
constexpr int kSteps[4] = {5, 9, 9, 9};       // K steps of 32 per layer
// packed B fragments: [layer][step][n-block][lane][8] bf16
constexpr int kPackOff[5] = {0, 5 * 2 * 64 * 8, 14 * 2 * 64 * 8, 23 * 2 * 64 * 8, 32 * 2 * 64 * 8};
constexpr int kPackElems = kPackOff[4];
constexpr int kBufX = (kR2 * kR2 * kCS > kR0 * kR0 * kCS0) ? kR2 * kR2 * kCS : kR0 * kR0 * kCS0;
constexpr int kBufY = kR1 * kR1 * kCS;
static_assert(kTO * kTO * 25 * 2 <= kBufX, "the output staging (FP32) must fit in buffer X");

struct PackedNet {
    bf16_t w[kPackElems];
    float bias[4][32];
};

// The B fragments and biases of one layer into registers (issued before the barrier that
// precedes the layer, so that their latency overlaps the wait).
template <int STEPS>
__device__ inline void load_layer(const PackedNet MG_G *pk, int layer, bf16x8 (&bw)[9][2], float &b0, float &b1)
{
    const int lane = threadIdx.x & 63;
    const bf16_t MG_G *wl = pk->w + kPackOff[layer];
#pragma unroll
    for (int s = 0; s < STEPS; ++s)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) bw[s][nb] = *(const bf16x8 MG_G *)(wl + ((s * 2 + nb) * 64 + lane) * 8);
    b0 = pk->bias[layer][lane % 16];
    b1 = pk->bias[layer][16 + lane % 16];
}

// One layer: out(region Wo x Wo, origin (gy0, gx0)) = conv(in(region Wo+2)), input channel
// stride CSin.  Each lane's A fragments sit at constant offsets from one LDS address per block.
template <int STEPS, int Wo, int CSin, bool FIRST, bool LAST>
__device__ inline void conv_layer(const bf16_t *in, bf16_t *out_bf, float *out_f, int gy0, int gx0, int n,
                                  const bf16x8 (&bw)[9][2], float b0, float b1)
{
    constexpr int Wi = Wo + 2, P = Wo * Wo, MB = (P + 15) / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4;
    // first layer: lane group g reads tap 2s + (g >> 1), channels 8 (g & 1) ..; other layers: tap s, channels 8 g ..
    const int cg = FIRST ? (g & 1) : g;
    const bool second_tap = FIRST && (g >> 1) != 0;
    // the whole region on the grid: no zero padding to apply (wave-uniform)
    const bool inside = gy0 >= 0 && gx0 >= 0 && gy0 + Wo <= n && gx0 + Wo <= n;
    for (int mb = wave; mb < MB; mb += kT / 64) {
        int pa = mb * 16 + (lane & 15);
        pa = pa < P ? pa : P - 1;
        const int oy = pa / Wo, ox = pa - oy * Wo;
        const bf16_t *base = in + (oy * Wi + ox) * CSin + cg * 8;
        f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < STEPS; ++s) {
            bf16x8 a;
            if (FIRST) {
                const int t0 = 2 * s, t1 = 2 * s + 1;
                const int off0 = ((t0 / 3) * Wi + t0 % 3) * CSin;
                if (t1 > 8) {
                    a = *(const bf16x8 *)(base + off0);
                    if (second_tap) a = bf16x8{};  // the padded tenth tap
                } else {
                    const int off1 = ((t1 / 3) * Wi + t1 % 3) * CSin;
                    a = *(const bf16x8 *)(base + off0 + (second_tap ? off1 - off0 : 0));
                }
            } else {
                a = *(const bf16x8 *)(base + ((s / 3) * Wi + s % 3) * CSin);
            }
            acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[s][0], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[s][1], acc1, 0, 0, 0);
        }
        const int pix0 = mb * 16 + 4 * g;
        if (LAST) {
            // staging [pixel][25] in FP32
            const int co0 = lane & 15, co1 = 16 + (lane & 15);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (pix0 + i >= P) continue;
                out_f[(pix0 + i) * 25 + co0] = acc0[i] + b0;
                if (co1 < 25) out_f[(pix0 + i) * 25 + co1] = acc1[i] + b1;
            }
            continue;
        }
        bf16_t *o = out_bf + pix0 * kCS + (lane & 15);
        if (inside && pix0 + 3 < P) {
            // ReLU only
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                o[i * kCS] = f32_to_bf16(fmaxf(acc0[i] + b0, 0.f));
                o[i * kCS + 16] = f32_to_bf16(fmaxf(acc1[i] + b1, 0.f));
            }
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int pix = pix0 + i;
                if (pix >= P) continue;
                const int py = pix / Wo, px = pix - py * Wo;
                const int gy = gy0 + py, gx = gx0 + px;
                const bool in_grid = gy >= 0 && gy < n && gx >= 0 && gx < n;
                const float v0 = acc0[i] + b0, v1 = acc1[i] + b1;
                o[i * kCS] = f32_to_bf16((in_grid && v0 > 0.f) ? v0 : 0.f);  // ReLU and zero padding off the grid
                o[i * kCS + 16] = f32_to_bf16((in_grid && v1 > 0.f) ? v1 : 0.f);
            }
        }
    }
}

// The whole network on the tile at (X0, Y0) of one level.
__device__ inline void cnn_tile(int n, int P, int64_t plane, const float MG_G *A32, const PackedNet MG_G *pk,
                                float omega, bf16_t MG_G *H, int X0, int Y0)
{
    __shared__ __align__(16) bf16_t bufX[kBufX];
    __shared__ __align__(16) bf16_t bufY[kBufY];
    __shared__ float sInv[kTO * kTO];      // 1 / a_C on the tile
    __shared__ bool sDiff[kTO * kTO];      // the row is a diffusion row (see below)
    const int tid = threadIdx.x;
    bf16x8 bw[9][2];
    float b0, b1;
    load_layer<5>(pk, 0, bw, b0, b1);
    // network input x0 = A / a_C on the tile plus a halo of four (zero off the grid); on the
    // tile itself also 1 / a_C and the row kind for the last step
    for (int q = tid; q < kR0 * kR0; q += kT) {
        const int gy = Y0 - 4 + q / kR0, gx = X0 - 4 + q % kR0;
        const bool ok = gy >= 0 && gy < n && gx >= 0 && gx < n;
        const int64_t p = ok ? (int64_t)gy * P + gx : 0;
        float a[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) a[c] = A32[c * plane + p];
        const float inv = 1.0f / a[kCentre];
#pragma unroll
        for (int c = 0; c < 16; ++c) bufX[q * kCS0 + c] = f32_to_bf16((ok && c < 9) ? a[c < 9 ? c : 0] * inv : 0.0f);
        const int ty = q / kR0 - 4, tx = q % kR0 - 4;
        if (ty >= 0 && ty < kTO && tx >= 0 && tx < kTO) {
            // a diffusion row's off-centre entries sum to a negative value; other rows (Dirichlet nodes
            // of a masked domain and their Galerkin images) take damped Jacobi.  Summed in channel order.
            float off = 0.f;
#pragma unroll
            for (int c = 0; c < 9; ++c)
                if (c != kCentre) off += a[c];
            sInv[ty * kTO + tx] = inv;
            sDiff[ty * kTO + tx] = off < 0.f;
        }
    }
    __syncthreads();
    conv_layer<5, kR1, kCS0, true, false>(bufX, bufY, nullptr, Y0 - 3, X0 - 3, n, bw, b0, b1);
    load_layer<9>(pk, 1, bw, b0, b1);
    __syncthreads();
    conv_layer<9, kR2, kCS, false, false>(bufY, bufX, nullptr, Y0 - 2, X0 - 2, n, bw, b0, b1);
    load_layer<9>(pk, 2, bw, b0, b1);
    __syncthreads();
    conv_layer<9, kR3, kCS, false, false>(bufX, bufY, nullptr, Y0 - 1, X0 - 1, n, bw, b0, b1);
    load_layer<9>(pk, 3, bw, b0, b1);
    __syncthreads();
    float *stage = (float *)bufX;
    conv_layer<9, kTO, kCS, false, true>(bufY, nullptr, stage, Y0, X0, n, bw, b0, b1);
    __syncthreads();
    // H = (omega * delta_0 + y) / a_C, plane by plane: two threads per node, planes 0..12 and 13..24
    static_assert(kT == 2 * kTO * kTO, "two threads per output node");
    {
        const int q = tid % (kTO * kTO), k0 = tid < kTO * kTO ? 0 : 13, k1 = tid < kTO * kTO ? 13 : 25;
        const int gy = Y0 + q / kTO, gx = X0 + q % kTO;
        if (gy < n && gx < n) {
            const int64_t p = (int64_t)gy * P + gx;
            const float inv = sInv[q];
            const bool diffusion = sDiff[q];
            for (int k = k0; k < k1; ++k)
                H[k * plane + p] = f32_to_bf16(((diffusion ? stage[q * 25 + k] : 0.f) + (k == 12 ? omega : 0.f)) * inv);
        }
    }
}

// One launch for every level of every problem: block b takes tile
// b - tile0 of the level whose [tile0, tile0 + tiles) holds b (levels in
// launch order, largest first, so the small ones fill the tail).  With
// size_filter != 0 only the levels of that size are computed.  With map.count
// > 0 each level takes the network listed for its size (per-level networks in
// one launch instead of one launch per size).
__global__ void __launch_bounds__(kT) k_cnn_fused_levels(const CnnLevelDesc *desc, int ndesc, int size_filter,
                                                         const PackedNet *pkg, CnnNetMap map, float omega)
{
    const int b = blockIdx.x;
    int lo = 0, hi = ndesc - 1;  // last level with tile0 <= b
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (desc[mid].tile0 <= b) lo = mid; else hi = mid - 1;
    }
    const CnnLevelDesc L = desc[lo];
    if (size_filter != 0 && L.n != size_filter) return;
    for (int k = 0; k < map.count; ++k)  // uniform
        if (map.n[k] == L.n) pkg = (const PackedNet *)map.packed[k];
    const int t = b - L.tile0, tx = (L.n + kTO - 1) / kTO;
    cnn_tile(L.n, L.P, L.plane, L.A32, (const PackedNet MG_G *)pkg, omega, L.H, (t % tx) * kTO, (t / tx) * kTO);
}

// Packs FP32 weights [Cout][Cin][3][3] + bias per layer into the per-lane
// B fragments and padded biases used by k_cnn_fused.
__global__ void k_pack(const float *params, PackedNet *pk)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int ch[5] = {9, 32, 32, 32, 25};
    if (idx < kPackElems) {
        int l = 0;
        while (idx >= kPackOff[l + 1]) ++l;
        int64_t woff = 0;
        for (int q = 0; q < l; ++q) woff += (int64_t)ch[q + 1] * ch[q] * 9 + ch[q + 1];
        const int cin = ch[l], cout = ch[l + 1];
        const int r = idx - kPackOff[l];
        const int e = r & 7, lane = (r >> 3) & 63, nb = (r >> 9) & 1, s = r >> 10;
        const int co = nb * 16 + (lane & 15), g = lane >> 4;
        int tap, ci;
        if (l == 0) {
            tap = 2 * s + (g >> 1);
            ci = 8 * (g & 1) + e;
        } else {
            tap = s;
            ci = 8 * g + e;
        }
        const bool ok = tap < 9 && ci < cin && co < cout;
        pk->w[idx] = f32_to_bf16(ok ? params[woff + ((int64_t)co * cin + ci) * 9 + tap] : 0.0f);
    }
    if (idx < 128) {
        const int l = idx / 32, co = idx % 32;
        int64_t woff = 0;
        for (int q = 0; q < l; ++q) woff += (int64_t)ch[q + 1] * ch[q] * 9 + ch[q + 1];
        const int64_t boff = woff + (int64_t)ch[l + 1] * ch[l] * 9;
        pk->bias[l][co] = co < ch[l + 1] ? params[boff + co] : 0.0f;
    }
}

}  // namespace

size_t packed_net_bytes() { return sizeof(PackedNet); }

void launch_pack_weights_mfma(const float *params, void *packed, hipStream_t st)
{
    k_pack<<<(kPackElems + 255) / 256, 256, 0, st>>>(params, (PackedNet *)packed);
}

int cnn_level_tiles(int n) { return ((n + kTO - 1) / kTO) * ((n + kTO - 1) / kTO); }

void launch_cnn_fused_levels(const CnnLevelDesc *desc, int ndesc, int total_tiles, int size_filter, const void *packed,
                             const CnnNetMap &map, double omega, hipStream_t st)
{
    if (ndesc < 1 || total_tiles < 1) return;
    k_cnn_fused_levels<<<total_tiles, kT, 0, st>>>(desc, ndesc, size_filter, (const PackedNet *)packed, map,
                                                   (float)omega);
}

}  // namespace mg
