// Training-step data structures and kernel launchers.
#pragma once
#include "common.hpp"

namespace mg {

// One problem of a training batch.  Planes have pitch n (no padding).
struct TrainProb {
    int index;        // position in the batch
    int n;
    int64_t plane;    // n * n
    const double MG_G *A;  // stencil [9][n][n] FP64 (caller's)
    const float MG_G *V;   // HF vectors [J][n][n] (caller's)
    float MG_G *x0;        // network input [9][plane]
    float MG_G *act;       // post-ReLU activations of layers 1..3, [3][32][plane]
    float MG_G *y;         // last-layer output [25][plane]
    float MG_G *Av;        // [J][plane]
    float MG_G *g;         // v - H A v, [J][plane]
    float MG_G *gnorm;     // [J]
    float MG_G *dA;        // gradient ping-pong buffers, [32][plane] each
    float MG_G *dB;
};

// Offsets of one layer's weights and bias in the flat parameter vector.
struct TrainLayer {
    int cin, cout;
    int64_t woff, boff;
};

void launch_tr_input(const TrainProb *probs, int nb, int n, hipStream_t st);
void launch_tr_conv_fwd(const TrainProb *probs, int nb, int n, const float *params, TrainLayer L, int layer,
                        hipStream_t st);
void launch_tr_av(const TrainProb *probs, int nb, int n, int J, hipStream_t st);
void launch_tr_residual_norm(const TrainProb *probs, int nb, int J, float omega, float *loss_part, hipStream_t st);
void launch_tr_dout(const TrainProb *probs, int nb, int n, int J, float scale, hipStream_t st);
// dL/dy copied from P.V ([25][plane] per problem), for a loss computed elsewhere
void launch_tr_dout_ext(const TrainProb *probs, int nb, int n, hipStream_t st);
void launch_tr_conv_bwd_data(const TrainProb *probs, int nb, int n, const float *params, TrainLayer L, int layer,
                             hipStream_t st);
void launch_tr_conv_bwd_weight(const TrainProb *probs, int nb, TrainLayer L, int layer, float *wpart, int64_t np,
                               hipStream_t st);
void launch_tr_reduce(const float *wpart, int B, int64_t np, float *grad, hipStream_t st);
void launch_tr_loss(const float *loss_part, int count, float scale, float *loss, hipStream_t st);
void launch_adam(int64_t np, float *p, float *m, float *v, const float *g, float lr, float b1, float b2, float eps,
                 float c1, float c2, hipStream_t st);
// Adam whose bias corrections come from the step number *t on the device.
void launch_adam_dev(int64_t np, float *p, float *m, float *v, const float *g, float lr, float b1, float b2,
                     float eps, const int64_t *t, hipStream_t st);
// dst[z][j] = pool[index[z J + j]] for count problems of size n (FP32 vectors of n * n).
void launch_tr_gather(int n, int count, int J, const float *pool, const int *index, float *dst, hipStream_t st);

}  // namespace mg

namespace mg {

// BF16 training path (train_mfma.hip): channel-last activations.
// Weight gradients are summed over groups of kTileGroup consecutive 16 x 16 tiles of one problem per
// workgroup (the convolutions keep one tile per workgroup: more workgroups in flight).
constexpr int kTileGroup = 4;
inline int trb_tile_groups(int n)
{
    const int t = (n + 15) / 16;
    return (t * t + kTileGroup - 1) / kTileGroup;
}
enum { kTbX0 = 0, kTbAct0 = 1, kTbAct1 = 2, kTbAct2 = 3, kTbDA = 4, kTbDB = 5 };

struct TrainProbB {
    int index;             // position in the batch
    int n;
    int64_t plane;         // n * n
    int part0;             // first weight-gradient part of this problem (one per tile group)
    const double MG_G *A;  // stencil [9][n][n] FP64 (caller's)
    const float MG_G *V;   // HF vectors [J][n][n] (caller's)
    bf16_t MG_G *x0;       // [plane][16]
    bf16_t MG_G *act;      // [3][plane][32], post-ReLU
    float MG_G *y;         // last layer output [plane][32]
    bf16_t MG_G *dA;       // gradient ping-pong, [plane][32] each
    bf16_t MG_G *dB;
    float MG_G *Av;        // [J][plane]
    float MG_G *g;         // [J][plane]
    float MG_G *gnorm;     // [J]
};

// Per-lane B fragments of every layer (forward; transposed and flipped for the data gradient of
// layers 1..3, bwd[0] unused) and the biases padded to 32, in one launch.
struct TrbPackJobs {
    TrainLayer layer[4];
    bf16_t *fwd[4], *bwd[4];
    float *bias[4];
};
void launch_trb_pack_all(const float *params, const TrbPackJobs &jobs, hipStream_t st);
void launch_trb_input(const TrainProbB *probs, int nb, int n, hipStream_t st);
void launch_trb_conv_fwd(const TrainProbB *probs, int nb, int n, int layer, const bf16_t *wpack, const float *bias,
                         hipStream_t st);
void launch_trb_conv_bwd_data(const TrainProbB *probs, int nb, int n, int layer, const bf16_t *wpack_t,
                              hipStream_t st);
void launch_trb_wgrad(const TrainProbB *probs, int nb, int n, int layer, int cout, float *part, hipStream_t st);
// part2: trb_reduce_scratch_bytes() of scratch for the per-slice sums
void launch_trb_reduce(const float *part, int ntiles, int cin, int cout, int64_t woff, int64_t boff, float *grad,
                       float *part2, hipStream_t st);
size_t trb_reduce_scratch_bytes();
void launch_trb_av(const TrainProbB *probs, int nb, int n, int J, hipStream_t st);
// part: FP64 [problems][nblk][J] block sums, nblk = trb_residual_blocks(largest n) (problem = TrainProbB.index)
void launch_trb_residual_norm(const TrainProbB *probs, int nb, int n, int J, float omega, float *loss_part,
                              double *part, int nblk, hipStream_t st);
int trb_residual_blocks(int nmax);
void launch_trb_dout(const TrainProbB *probs, int nb, int n, int J, float scale, hipStream_t st);

}  // namespace mg
