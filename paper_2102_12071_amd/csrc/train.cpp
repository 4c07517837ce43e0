// Training step driver for the high-frequency smoothing loss: groups the
// batch by grid size and runs forward, loss, backward and Adam on the device,
// either in FP32 on the vector units (precision 0, the parity path) or in
// BF16 on the matrix cores with FP32 accumulation (precision 1).
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.hpp"
#include "train.hpp"

using namespace mg;

namespace {

struct Layout {
    size_t bytes = 0;
    size_t take(size_t b)
    {
        size_t off = bytes;
        bytes += (b + 255) & ~(size_t)255;
        return off;
    }
};

struct Cls {
    int first, count, n;
};

// Problem order grouped by size, and the resulting size classes.
void classes_of(const mg_train_batch *b, std::vector<int> &order, std::vector<Cls> &classes)
{
    const int B = b->nprob;
    order.resize(B);
    for (int q = 0; q < B; ++q) order[q] = q;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b->n[x] < b->n[y]; });
    classes.clear();
    for (int k = 0; k < B;) {
        int e = k;
        while (e < B && b->n[order[e]] == b->n[order[k]]) ++e;
        classes.push_back({k, e - k, b->n[order[k]]});
        k = e;
    }
}

void layer_offsets(const mg_net_s &net, TrainLayer layers[4])
{
    int64_t woff = 0;
    for (int l = 0; l < 4; ++l) {
        layers[l].cin = net.ch[l];
        layers[l].cout = net.ch[l + 1];
        layers[l].woff = woff;
        layers[l].boff = woff + (int64_t)layers[l].cout * layers[l].cin * 9;
        woff = layers[l].boff + layers[l].cout;
    }
}

mg_status ensure_scratch(mg_net_s &net, size_t bytes)
{
    // the previous step may still use the scratch and the descriptor upload's source
    MG_HIP(hipStreamSynchronize(net.join.internal));
    if (bytes > net.scratch_bytes) {
        net.scratch.release();
        net.scratch_bytes = 0;
        MG_TRY(net.scratch.alloc(&net.scratch_base, bytes));
        net.scratch_bytes = bytes;
    }
    return MG_OK;
}

template <typename D>
mg_status upload_desc(mg_net_s &net, const std::vector<D> &desc, D *d_desc, hipStream_t st)
{
    // the upload's source must outlive the asynchronous copy: keep the bytes in the network object
    net.host_desc.assign((const char *)desc.data(), (const char *)(desc.data() + desc.size()));
    MG_HIP(hipMemcpyAsync(d_desc, net.host_desc.data(), sizeof(D) * desc.size(), hipMemcpyHostToDevice, st));
    return MG_OK;
}

// FP32 path: planar activations, direct convolutions.  ext: the output
// gradient dL/dy is given (b->vectors[q]: [25][n*n] per problem, nvec = 0)
// instead of coming from the high-frequency loss.
mg_status step_fp32(mg_net_s &net, const mg_train_batch *b, const mg_train_opts &o, float *loss_part, float *d_loss,
                    hipStream_t st, bool ext = false)
{
    const int B = b->nprob, J = b->nvec;
    Layout lay;
    std::vector<size_t> off(B);
    for (int q = 0; q < B; ++q) {
        const size_t v = (size_t)b->n[q] * b->n[q] * sizeof(float);
        off[q] = lay.take(v * (9 + 96 + 25 + 2 * J + 64) + J * sizeof(float));
    }
    const size_t off_desc = lay.take(sizeof(TrainProb) * B);
    const size_t off_wpart = lay.take(sizeof(float) * net.np * B);
    (void)off_wpart;
    char *base = (char *)net.scratch_base;
    std::vector<int> order;
    std::vector<Cls> classes;
    classes_of(b, order, classes);
    std::vector<TrainProb> desc(B);
    for (int k = 0; k < B; ++k) {
        const int q = order[k];
        const int n = b->n[q];
        const int64_t v = (int64_t)n * n;
        float *p = (float *)(base + off[q]);
        TrainProb &d = desc[k];
        d.index = q;
        d.n = n;
        d.plane = v;
        d.A = b->stencil[q];
        d.V = b->vectors[q];
        d.x0 = p;
        d.act = d.x0 + 9 * v;
        d.y = d.act + 96 * v;
        d.Av = d.y + 25 * v;
        d.g = d.Av + (int64_t)J * v;
        d.dA = d.g + (int64_t)J * v;
        d.dB = d.dA + 32 * v;
        d.gnorm = d.dB + 32 * v;
    }
    TrainLayer layers[4];
    layer_offsets(net, layers);
    TrainProb *d_desc = (TrainProb *)(base + off_desc);
    float *wpart = (float *)(base + off_wpart);
    MG_TRY(upload_desc(net, desc, d_desc, st));
    const float scale = J > 0 ? 1.0f / ((float)B * (float)J) : 0.0f;
    for (const Cls &c : classes) launch_tr_input(d_desc + c.first, c.count, c.n, st);
    for (int l = 0; l < 4; ++l)
        for (const Cls &c : classes) launch_tr_conv_fwd(d_desc + c.first, c.count, c.n, net.params, layers[l], l, st);
    for (const Cls &c : classes) {
        if (ext) {
            launch_tr_dout_ext(d_desc + c.first, c.count, c.n, st);
            continue;
        }
        launch_tr_av(d_desc + c.first, c.count, c.n, J, st);
        launch_tr_residual_norm(d_desc + c.first, c.count, J, (float)o.omega, loss_part, st);
        launch_tr_dout(d_desc + c.first, c.count, c.n, J, scale, st);
    }
    for (int l = 3; l >= 0; --l) {
        for (const Cls &c : classes) {
            launch_tr_conv_bwd_weight(d_desc + c.first, c.count, layers[l], l, wpart, net.np, st);
            if (l > 0) launch_tr_conv_bwd_data(d_desc + c.first, c.count, c.n, net.params, layers[l], l, st);
        }
    }
    launch_tr_reduce(wpart, B, net.np, net.grad, st);
    (void)d_loss;
    return MG_OK;
}

size_t fp32_scratch(const mg_net_s &net, const mg_train_batch *b)
{
    const int B = b->nprob, J = b->nvec;
    Layout lay;
    for (int q = 0; q < B; ++q) {
        const size_t v = (size_t)b->n[q] * b->n[q] * sizeof(float);
        lay.take(v * (9 + 96 + 25 + 2 * J + 64) + J * sizeof(float));
    }
    lay.take(sizeof(TrainProb) * B);
    lay.take(sizeof(float) * net.np * B);
    return lay.bytes;
}

// BF16 path: channel-last activations, MFMA convolutions.
struct Bf16Layout {
    std::vector<size_t> off;
    size_t desc, pack_fwd[4], pack_bwd[4], bias[4], part, part2, respart;
    int ntiles, resblk;
    size_t bytes;
};

Bf16Layout bf16_layout(const mg_train_batch *b)
{
    const int B = b->nprob, J = b->nvec;
    Bf16Layout L;
    Layout lay;
    L.off.resize(B);
    L.ntiles = 0;
    for (int q = 0; q < B; ++q) {
        const size_t v = (size_t)b->n[q] * b->n[q];
        L.off[q] = lay.take(v * (16 * 2 + 96 * 2 + 32 * 4 + 64 * 2 + 2 * J * 4) + J * sizeof(float));
        const int t = (b->n[q] + 15) / 16;
        L.ntiles += t * t;
    }
    L.desc = lay.take(sizeof(TrainProbB) * B);
    for (int l = 0; l < 4; ++l) {
        L.pack_fwd[l] = lay.take((l == 0 ? 5 : 9) * 2 * 64 * 8 * sizeof(bf16_t));
        L.pack_bwd[l] = lay.take(9 * 2 * 64 * 8 * sizeof(bf16_t));
        L.bias[l] = lay.take(32 * sizeof(float));
    }
    L.part = lay.take((size_t)L.ntiles * (9 * 32 * 32 + 32) * sizeof(float));
    L.part2 = lay.take(trb_reduce_scratch_bytes());
    int nmax = 0;
    for (int q = 0; q < B; ++q) nmax = std::max(nmax, (int)b->n[q]);
    L.resblk = trb_residual_blocks(nmax);
    L.respart = lay.take(sizeof(double) * (size_t)B * L.resblk * J);
    L.bytes = lay.bytes;
    return L;
}

mg_status step_bf16(mg_net_s &net, const mg_train_batch *b, const mg_train_opts &o, const Bf16Layout &L,
                    float *loss_part, hipStream_t st)
{
    const int B = b->nprob, J = b->nvec;
    char *base = (char *)net.scratch_base;
    std::vector<int> order;
    std::vector<Cls> classes;
    classes_of(b, order, classes);
    std::vector<TrainProbB> desc(B);
    int tile0 = 0;
    for (int k = 0; k < B; ++k) {
        const int q = order[k];
        const int n = b->n[q];
        const int64_t v = (int64_t)n * n;
        char *p = base + L.off[q];
        TrainProbB &d = desc[k];
        d.index = q;
        d.n = n;
        d.plane = v;
        d.tile0 = tile0;
        tile0 += ((n + 15) / 16) * ((n + 15) / 16);
        d.A = b->stencil[q];
        d.V = b->vectors[q];
        d.x0 = (bf16_t *)p;
        d.act = d.x0 + 16 * v;
        d.dA = d.act + 96 * v;
        d.dB = d.dA + 32 * v;
        d.y = (float *)(d.dB + 32 * v);
        d.Av = d.y + 32 * v;
        d.g = d.Av + (int64_t)J * v;
        d.gnorm = d.g + (int64_t)J * v;
    }
    TrainLayer layers[4];
    layer_offsets(net, layers);
    TrainProbB *d_desc = (TrainProbB *)(base + L.desc);
    float *part = (float *)(base + L.part);
    MG_TRY(upload_desc(net, desc, d_desc, st));
    bf16_t *pf[4], *pb[4];
    float *bias[4];
    for (int l = 0; l < 4; ++l) {
        pf[l] = (bf16_t *)(base + L.pack_fwd[l]);
        pb[l] = (bf16_t *)(base + L.pack_bwd[l]);
        bias[l] = (float *)(base + L.bias[l]);
        launch_trb_pack(net.params, layers[l].woff, layers[l].cin, layers[l].cout, l == 0, false, pf[l], st);
        if (l > 0) launch_trb_pack(net.params, layers[l].woff, layers[l].cin, layers[l].cout, false, true, pb[l], st);
        launch_trb_bias(net.params, layers[l].boff, layers[l].cout, bias[l], st);
    }
    const float scale = 1.0f / ((float)B * (float)J);
    for (const Cls &c : classes) launch_trb_input(d_desc + c.first, c.count, c.n, st);
    for (int l = 0; l < 4; ++l)
        for (const Cls &c : classes) launch_trb_conv_fwd(d_desc + c.first, c.count, c.n, l, pf[l], bias[l], st);
    for (const Cls &c : classes) {
        launch_trb_av(d_desc + c.first, c.count, c.n, J, st);
        launch_trb_residual_norm(d_desc + c.first, c.count, c.n, J, (float)o.omega, loss_part,
                                 (double *)(base + L.respart), L.resblk, st);
        launch_trb_dout(d_desc + c.first, c.count, c.n, J, scale, st);
    }
    for (int l = 3; l >= 0; --l) {
        for (const Cls &c : classes) launch_trb_wgrad(d_desc + c.first, c.count, c.n, l, layers[l].cout, part, st);
        launch_trb_reduce(part, L.ntiles, layers[l].cin, layers[l].cout, layers[l].woff, layers[l].boff, net.grad,
                          (float *)(base + L.part2), st);
        if (l > 0)
            for (const Cls &c : classes) launch_trb_conv_bwd_data(d_desc + c.first, c.count, c.n, l, pb[l], st);
    }
    return MG_OK;
}

}  // namespace

namespace mg {

mg_status net_backward_ext(mg_net_s &net, int B, const int *n, const double *const *stencil,
                           const float *const *dout, hipStream_t st)
{
    const mg_train_batch b{B, n, stencil, dout, 0};
    MG_TRY(ensure_scratch(net, fp32_scratch(net, &b)));
    mg_train_opts o;
    mg_train_opts_default(&o);
    return step_fp32(net, &b, o, nullptr, nullptr, st, true);
}

void net_adam(mg_net_s &net, const mg_train_opts &o, hipStream_t st)
{
    net.step += 1;
    const double t = (double)net.step;
    const float c1 = (float)(1.0 - std::pow((double)o.beta1, t));
    const float c2 = (float)(1.0 - std::pow((double)o.beta2, t));
    launch_adam(net.np, net.params, net.m, net.v, net.grad, o.lr, o.beta1, o.beta2, o.adam_eps, c1, c2, st);
    net.packed_valid = false;
}

mg_status check_train_opts(const mg_train_opts &o)
{
    if (o.precision != 0 && o.precision != 1) return set_error(MG_ERR_ARG, "training precision must be 0 or 1");
    if (!(o.lr >= 0.0f) || !(o.beta1 >= 0.0f && o.beta1 < 1.0f) || !(o.beta2 >= 0.0f && o.beta2 < 1.0f))
        return set_error(MG_ERR_ARG, "bad Adam parameters");
    return MG_OK;
}

}  // namespace mg

extern "C" mg_status mg_train_step(mg_net net, const mg_train_batch *b, const mg_train_opts *o_in, float *loss,
                                   float *grad)
{
    clear_error();
    if (!net) return set_error(MG_ERR_ARG, "net is null");
    if (!b || b->nprob < 1 || !b->n || !b->stencil || !b->vectors || b->nvec < 1)
        return set_error(MG_ERR_ARG, "batch needs nprob >= 1, sizes, stencils, vectors and nvec >= 1");
    mg_train_opts o;
    if (o_in)
        o = *o_in;
    else
        mg_train_opts_default(&o);
    MG_TRY(check_train_opts(o));
    const int B = b->nprob, J = b->nvec;
    for (int q = 0; q < B; ++q) {
        const int n = b->n[q];
        if (n < 3 || n > 255 || (n & 1) == 0) return set_error(MG_ERR_ARG, "problem %d: n = %d must be odd in [3, 255]", q, n);
        if (!b->stencil[q] || !b->vectors[q]) return set_error(MG_ERR_ARG, "problem %d: null pointer", q);
    }
    Bf16Layout L16;
    size_t need = 0;
    if (o.precision == 1) {
        L16 = bf16_layout(b);
        need = L16.bytes;
    } else {
        need = fp32_scratch(*net, b);
    }
    const size_t loss_bytes = ((sizeof(float) * (B * J + 1)) + 255) & ~(size_t)255;
    MG_TRY(ensure_scratch(*net, need + loss_bytes));
    float *loss_part = (float *)((char *)net->scratch_base + need);
    float *d_loss = loss_part + B * J;
    MG_TRY(net->join.enter());
    hipStream_t st = net->join.internal;
    if (o.precision == 1)
        MG_TRY(step_bf16(*net, b, o, L16, loss_part, st));
    else
        MG_TRY(step_fp32(*net, b, o, loss_part, d_loss, st));
    const float scale = 1.0f / ((float)B * (float)J);
    launch_tr_loss(loss_part, B * J, scale, d_loss, st);
    if (o.apply_update) net_adam(*net, o, st);
    MG_HIP(hipGetLastError());
    if (loss || grad) {
        if (loss) MG_HIP(hipMemcpyAsync(loss, d_loss, sizeof(float), hipMemcpyDeviceToHost, st));
        if (grad) MG_HIP(hipMemcpyAsync(grad, net->grad, sizeof(float) * net->np, hipMemcpyDeviceToHost, st));
        MG_HIP(hipStreamSynchronize(st));
    }
    return net->join.leave();
}
