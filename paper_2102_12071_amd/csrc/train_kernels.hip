// Training kernels for the high-frequency smoothing loss (FP32 path):
//   forward of the stencil-to-smoother network with stored activations,
//   the loss L = 1/(B J) sum ||v - H A v|| and its gradient with respect to the
//   network output, reverse-mode convolution layers (data and weight
//   gradients, ReLU masks), a deterministic reduction over problems, and Adam.
// Problems of a batch are grouped by size; each launch covers one size class
// with blockIdx.z selecting the problem (and channel where noted).
#include "common.hpp"
#include "train.hpp"

namespace mg {

namespace {

constexpr int kT = 256;

__device__ inline bool inside(int n, int i, int j) { return i >= 0 && i < n && j >= 0 && j < n; }

// x0 = A / a_C from the FP64 stencil.
__global__ void __launch_bounds__(kT) k_tr_input(const TrainProb *probs)
{
    const TrainProb &P = probs[blockIdx.z];
    const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (p >= P.plane) return;
    const double ac = P.A[kCentre * P.plane + p];
    for (int c = 0; c < 9; ++c) P.x0[c * P.plane + p] = (float)(P.A[c * P.plane + p] / ac);
}

__device__ inline const float MG_G *layer_input(const TrainProb &P, int l)
{
    return l == 0 ? P.x0 : P.act + (int64_t)(l - 1) * 32 * P.plane;
}

// out[co] = b[co] + sum_ci sum_tap w[co][ci][tap] in[ci](p + tap - 1); ReLU for l < 3.
// grid.z = problem * cout + co.
__global__ void __launch_bounds__(kT) k_tr_conv_fwd(const TrainProb *probs, const float *params, TrainLayer L,
                                                    int layer)
{
    const int bz = blockIdx.z / L.cout, co = blockIdx.z % L.cout;
    const TrainProb &P = probs[bz];
    const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (p >= P.plane) return;
    const int n = P.n, i = (int)(p % n), j = (int)(p / n);
    const float MG_G *in = layer_input(P, layer);
    const float *w = params + L.woff + (int64_t)co * L.cin * 9;
    float acc = params[L.boff + co];
    for (int ci = 0; ci < L.cin; ++ci) {
        const float MG_G *x = in + (int64_t)ci * P.plane;
        const float *wk = w + ci * 9;
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int ii = i + t % 3 - 1, jj = j + t / 3 - 1;
            if (inside(n, ii, jj)) acc += wk[t] * x[(int64_t)jj * n + ii];
        }
    }
    if (layer < 3) {
        acc = acc > 0.0f ? acc : 0.0f;
        P.act[((int64_t)layer * 32 + co) * P.plane + p] = acc;
    } else {
        P.y[(int64_t)co * P.plane + p] = acc;
    }
}

// Av_j = A v_j (FP32 arithmetic on the FP64 stencil).  grid.z = problem * J + j.
__global__ void __launch_bounds__(kT) k_tr_av(const TrainProb *probs, int J)
{
    const TrainProb &P = probs[blockIdx.z / J];
    const int jv = blockIdx.z % J;
    const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (p >= P.plane) return;
    const int n = P.n, i = (int)(p % n), j = (int)(p / n);
    const float MG_G *v = P.V + (int64_t)jv * P.plane;
    float acc = 0.0f;
#pragma unroll
    for (int c = 0; c < 9; ++c) {
        const int ii = i + c % 3 - 1, jj = j + c / 3 - 1;
        if (inside(n, ii, jj)) acc += (float)P.A[c * P.plane + p] * v[(int64_t)jj * n + ii];
    }
    P.Av[(int64_t)jv * P.plane + p] = acc;
}

// g_j = v_j - H A v_j with (H x)_p = (1/a_C) sum_k W_p[k] x_{p+k}, W = omega*delta_0 + y;
// one block per (problem, vector); writes g and ||g_j||.
__global__ void __launch_bounds__(kT) k_tr_residual_norm(const TrainProb *probs, int J, float omega, float *loss_part)
{
    __shared__ double red[kT / 64];
    const TrainProb &P = probs[blockIdx.x / J];
    const int jv = blockIdx.x % J;
    const int n = P.n;
    const float MG_G *Av = P.Av + (int64_t)jv * P.plane;
    const float MG_G *v = P.V + (int64_t)jv * P.plane;
    float MG_G *g = P.g + (int64_t)jv * P.plane;
    double acc2 = 0.0;
    for (int64_t p = threadIdx.x; p < P.plane; p += kT) {
        const int i = (int)(p % n), j = (int)(p / n);
        float y = 0.0f;
        for (int k = 0; k < 25; ++k) {
            const int ii = i + k % 5 - 2, jj = j + k / 5 - 2;
            if (!inside(n, ii, jj)) continue;
            const float wk = P.y[(int64_t)k * P.plane + p] + (k == 12 ? omega : 0.0f);
            y += wk * Av[(int64_t)jj * n + ii];
        }
        y /= (float)P.A[kCentre * P.plane + p];
        const float gv = v[p] - y;
        g[p] = gv;
        acc2 += (double)gv * gv;
    }
    const double s = block_sum<kT>(acc2, red);
    if (threadIdx.x == 0) {
        const float gn = (float)sqrt(s);
        P.gnorm[jv] = gn;
        loss_part[P.index * J + jv] = gn;
    }
}

// dL/dW_p[k] = -(1/(B J)) sum_j (g_j(p) / ||g_j||) Av_j(p + k) / a_C(p), written to dA.
__global__ void __launch_bounds__(kT) k_tr_dout(const TrainProb *probs, int J, float scale)
{
    const TrainProb &P = probs[blockIdx.z];
    const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (p >= P.plane) return;
    const int n = P.n, i = (int)(p % n), j = (int)(p / n);
    const float inv_ac = 1.0f / (float)P.A[kCentre * P.plane + p];
    float acc[25];
#pragma unroll
    for (int k = 0; k < 25; ++k) acc[k] = 0.0f;
    for (int jv = 0; jv < J; ++jv) {
        const float gn = P.gnorm[jv];
        if (gn == 0.0f) continue;
        const float c = -scale * P.g[(int64_t)jv * P.plane + p] / gn * inv_ac;
        const float MG_G *Av = P.Av + (int64_t)jv * P.plane;
#pragma unroll
        for (int k = 0; k < 25; ++k) {
            const int ii = i + k % 5 - 2, jj = j + k / 5 - 2;
            if (inside(n, ii, jj)) acc[k] += c * Av[(int64_t)jj * n + ii];
        }
    }
#pragma unroll
    for (int k = 0; k < 25; ++k) P.dA[(int64_t)k * P.plane + p] = acc[k];
}

// Output gradient given from outside (another loss): dL/dy = the 25 planes at P.V.
__global__ void __launch_bounds__(kT) k_tr_dout_ext(const TrainProb *probs)
{
    const TrainProb &P = probs[blockIdx.z];
    const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (p >= P.plane) return;
#pragma unroll
    for (int k = 0; k < 25; ++k) P.dA[(int64_t)k * P.plane + p] = P.V[(int64_t)k * P.plane + p];
}

__device__ inline float MG_G *dpre_buf(const TrainProb &P, int layer) { return (layer & 1) ? P.dA : P.dB; }

// dX[ci](q) = sum_co sum_tap w[co][ci][tap] dPre[co](q - tap + 1), masked by the
// previous layer's ReLU (act > 0).  grid.z = problem * cin + ci.
__global__ void __launch_bounds__(kT) k_tr_conv_bwd_data(const TrainProb *probs, const float *params, TrainLayer L,
                                                         int layer)
{
    const int bz = blockIdx.z / L.cin, ci = blockIdx.z % L.cin;
    const TrainProb &P = probs[bz];
    const int64_t q = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (q >= P.plane) return;
    const int n = P.n, i = (int)(q % n), j = (int)(q / n);
    const float MG_G *dp = (layer == 3) ? P.dA : dpre_buf(P, layer);
    float acc = 0.0f;
    for (int co = 0; co < L.cout; ++co) {
        const float *w = params + L.woff + ((int64_t)co * L.cin + ci) * 9;
        const float MG_G *d = dp + (int64_t)co * P.plane;
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int ii = i - (t % 3 - 1), jj = j - (t / 3 - 1);  // output node that read q through tap t
            if (inside(n, ii, jj)) acc += w[t] * d[(int64_t)jj * n + ii];
        }
    }
    const float a = P.act[((int64_t)(layer - 1) * 32 + ci) * P.plane + q];
    float MG_G *out = dpre_buf(P, layer - 1);
    out[(int64_t)ci * P.plane + q] = a > 0.0f ? acc : 0.0f;
}

// Per-problem weight and bias gradient of one layer:
//   gw[co][ci][tap] = sum_p dPre[co](p) X[ci](p + tap - 1),  gb[co] = sum_p dPre[co](p).
// One block per problem; thread t owns input channel ci = t % cin and the
// output channels co = t / cin + k * (kT / cin).  Rows are staged in LDS.
constexpr int kMaxRow = 256;
__global__ void __launch_bounds__(kT) k_tr_conv_bwd_weight(const TrainProb *probs, TrainLayer L, int layer,
                                                           float *wpart, int64_t np)
{
    __shared__ float xs[3][32][kMaxRow + 2];  // input rows j-1, j, j+1 with one halo column each side
    __shared__ float ds[32][kMaxRow];         // dPre row j
    const TrainProb &P = probs[blockIdx.z];
    const int n = P.n;
    const float MG_G *X = layer_input(P, layer);
    const float MG_G *dp = (layer == 3) ? P.dA : dpre_buf(P, layer);
    const int t = threadIdx.x;
    const int groups = kT / L.cin;
    const int ci = t % L.cin, g0 = t / L.cin;
    const bool active = t < groups * L.cin;
    float acc[4][9];
    float bacc = 0.0f;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int q = 0; q < 9; ++q) acc[a][q] = 0.0f;
    for (int j = 0; j < n; ++j) {
        __syncthreads();
        for (int e = t; e < 3 * L.cin * (n + 2); e += kT) {
            const int r = e / (L.cin * (n + 2)), rem = e % (L.cin * (n + 2));
            const int c = rem / (n + 2), x = rem % (n + 2) - 1;
            const int jj = j + r - 1;
            xs[r][c][x + 1] = inside(n, x, jj) ? X[(int64_t)c * P.plane + (int64_t)jj * n + x] : 0.0f;
        }
        for (int e = t; e < L.cout * n; e += kT) {
            const int c = e / n, x = e % n;
            ds[c][x] = dp[(int64_t)c * P.plane + (int64_t)j * n + x];
        }
        __syncthreads();
        if (!active) continue;
        for (int x = 0; x < n; ++x) {
            float xv[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) xv[q] = xs[q / 3][ci][x + q % 3];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const int co = g0 + a * groups;
                if (co >= L.cout) break;
                const float d = ds[co][x];
#pragma unroll
                for (int q = 0; q < 9; ++q) acc[a][q] += d * xv[q];
            }
        }
        if (t < L.cout)
            for (int x = 0; x < n; ++x) bacc += ds[t][x];
    }
    float *out = wpart + (int64_t)P.index * np;
    if (active) {
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int co = g0 + a * groups;
            if (co >= L.cout) break;
#pragma unroll
            for (int q = 0; q < 9; ++q) out[L.woff + ((int64_t)co * L.cin + ci) * 9 + q] = acc[a][q];
        }
    }
    if (t < L.cout) out[L.boff + t] = bacc;
}

// grad[q] = sum_b wpart[b][q] in problem order; loss = sum_{b,j} loss_part / (B J).
__global__ void __launch_bounds__(kT) k_tr_reduce(const float *wpart, int B, int64_t np, float *grad)
{
    const int64_t q = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (q >= np) return;
    float s = 0.0f;
    for (int b = 0; b < B; ++b) s += wpart[(int64_t)b * np + q];
    grad[q] = s;
}

__global__ void __launch_bounds__(kT) k_tr_loss(const float *loss_part, int count, float scale, float *loss)
{
    __shared__ double red[kT / 64];
    double s = 0.0;
    for (int q = threadIdx.x; q < count; q += kT) s += loss_part[q];
    s = block_sum<kT>(s, red);
    if (threadIdx.x == 0) *loss = (float)(s * scale);
}

// Adam with bias correction, FP32 master weights (PyTorch's formulation).
__global__ void __launch_bounds__(kT) k_adam(int64_t np, float *p, float *m, float *v, const float *g, float lr,
                                             float b1, float b2, float eps, float c1, float c2)
{
    const int64_t q = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (q >= np) return;
    const float gq = g[q];
    const float mq = b1 * m[q] + (1.0f - b1) * gq;
    const float vq = b2 * v[q] + (1.0f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    const float mhat = mq / c1, vhat = vq / c2;
    p[q] -= lr * mhat / (sqrtf(vhat) + eps);
}

// Adam with the bias corrections of step *t (device): the step a captured graph replays.
__global__ void __launch_bounds__(kT) k_adam_dev(int64_t np, float *p, float *m, float *v, const float *g, float lr,
                                                 float b1, float b2, float eps, const int64_t *t)
{
    const int64_t q = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (q >= np) return;
    const double td = (double)*t;
    const float c1 = (float)(1.0 - pow((double)b1, td)), c2 = (float)(1.0 - pow((double)b2, td));
    const float gq = g[q];
    const float mq = b1 * m[q] + (1.0f - b1) * gq;
    const float vq = b2 * v[q] + (1.0f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    const float mhat = mq / c1, vhat = vq / c2;
    p[q] -= lr * mhat / (sqrtf(vhat) + eps);
}

// dst[z][j] = pool[index[z * J + j]] for the count problems of one size (vectors of n * n FP32).
__global__ void __launch_bounds__(kT) k_tr_gather(int64_t nn, int J, const float *pool, const int *index, float *dst)
{
    const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (p >= nn) return;
    const int j = blockIdx.y, z = blockIdx.z;
    dst[((int64_t)z * J + j) * nn + p] = pool[(int64_t)index[z * J + j] * nn + p];
}

inline unsigned blocks_for(int64_t count) { return (unsigned)((count + kT - 1) / kT); }

}  // namespace

void launch_tr_input(const TrainProb *probs, int nb, int n, hipStream_t st)
{
    k_tr_input<<<dim3(blocks_for((int64_t)n * n), 1, nb), kT, 0, st>>>(probs);
}

void launch_tr_conv_fwd(const TrainProb *probs, int nb, int n, const float *params, TrainLayer L, int layer,
                        hipStream_t st)
{
    k_tr_conv_fwd<<<dim3(blocks_for((int64_t)n * n), 1, nb * L.cout), kT, 0, st>>>(probs, params, L, layer);
}

void launch_tr_av(const TrainProb *probs, int nb, int n, int J, hipStream_t st)
{
    k_tr_av<<<dim3(blocks_for((int64_t)n * n), 1, nb * J), kT, 0, st>>>(probs, J);
}

void launch_tr_residual_norm(const TrainProb *probs, int nb, int J, float omega, float *loss_part, hipStream_t st)
{
    k_tr_residual_norm<<<nb * J, kT, 0, st>>>(probs, J, omega, loss_part);
}

void launch_tr_dout(const TrainProb *probs, int nb, int n, int J, float scale, hipStream_t st)
{
    k_tr_dout<<<dim3(blocks_for((int64_t)n * n), 1, nb), kT, 0, st>>>(probs, J, scale);
}

void launch_tr_dout_ext(const TrainProb *probs, int nb, int n, hipStream_t st)
{
    k_tr_dout_ext<<<dim3(blocks_for((int64_t)n * n), 1, nb), kT, 0, st>>>(probs);
}

void launch_tr_conv_bwd_data(const TrainProb *probs, int nb, int n, const float *params, TrainLayer L, int layer,
                             hipStream_t st)
{
    k_tr_conv_bwd_data<<<dim3(blocks_for((int64_t)n * n), 1, nb * L.cin), kT, 0, st>>>(probs, params, L, layer);
}

void launch_tr_conv_bwd_weight(const TrainProb *probs, int nb, TrainLayer L, int layer, float *wpart, int64_t np,
                               hipStream_t st)
{
    k_tr_conv_bwd_weight<<<dim3(1, 1, nb), kT, 0, st>>>(probs, L, layer, wpart, np);
}

void launch_tr_reduce(const float *wpart, int B, int64_t np, float *grad, hipStream_t st)
{
    k_tr_reduce<<<blocks_for(np), kT, 0, st>>>(wpart, B, np, grad);
}

void launch_tr_loss(const float *loss_part, int count, float scale, float *loss, hipStream_t st)
{
    k_tr_loss<<<1, kT, 0, st>>>(loss_part, count, scale, loss);
}

void launch_adam_dev(int64_t np, float *p, float *m, float *v, const float *g, float lr, float b1, float b2,
                     float eps, const int64_t *t, hipStream_t st)
{
    k_adam_dev<<<blocks_for(np), kT, 0, st>>>(np, p, m, v, g, lr, b1, b2, eps, t);
}

void launch_tr_gather(int n, int count, int J, const float *pool, const int *index, float *dst, hipStream_t st)
{
    const int64_t nn = (int64_t)n * n;
    k_tr_gather<<<dim3(blocks_for(nn), J, count), kT, 0, st>>>(nn, J, pool, index, dst);
}

void launch_adam(int64_t np, float *p, float *m, float *v, const float *g, float lr, float b1, float b2, float eps,
                 float c1, float c2, hipStream_t st)
{
    k_adam<<<blocks_for(np), kT, 0, st>>>(np, p, m, v, g, lr, b1, b2, eps, c1, c2);
}

}  // namespace mg
