// Training step driver for the high-frequency smoothing loss: groups the
// batch by grid size, runs forward, loss, backward and Adam on the device.
#include <algorithm>
#include <cmath>
#include <map>
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

}  // namespace

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
    if (o.precision != 0) return set_error(MG_ERR_ARG, "training precision must be 0 (FP32) in this build");
    if (!(o.lr >= 0.0f) || !(o.beta1 >= 0.0f && o.beta1 < 1.0f) || !(o.beta2 >= 0.0f && o.beta2 < 1.0f))
        return set_error(MG_ERR_ARG, "bad Adam parameters");
    const int B = b->nprob, J = b->nvec;
    for (int q = 0; q < B; ++q) {
        const int n = b->n[q];
        if (n < 3 || n > 255 || (n & 1) == 0) return set_error(MG_ERR_ARG, "problem %d: n = %d must be odd in [3, 255]", q, n);
        if (!b->stencil[q] || !b->vectors[q]) return set_error(MG_ERR_ARG, "problem %d: null pointer", q);
    }
    // scratch layout: per-problem buffers, descriptors, partial gradients, loss parts
    Layout lay;
    std::vector<size_t> off(B);
    for (int q = 0; q < B; ++q) {
        const size_t v = (size_t)b->n[q] * b->n[q] * sizeof(float);
        off[q] = lay.take(v * (9 + 96 + 25 + 2 * J + 64) + J * sizeof(float));
    }
    const size_t off_desc = lay.take(sizeof(TrainProb) * B);
    const size_t off_wpart = lay.take(sizeof(float) * net->np * B);
    const size_t off_loss = lay.take(sizeof(float) * (B * J + 1));
    // the previous step may still use the scratch and the descriptor upload's source
    MG_HIP(hipStreamSynchronize(net->join.internal));
    if (lay.bytes > net->scratch_bytes) {
        net->scratch.release();
        net->scratch_bytes = 0;
        MG_TRY(net->scratch.alloc(&net->scratch_base, lay.bytes));
        net->scratch_bytes = lay.bytes;
    }
    char *base = (char *)net->scratch_base;
    // descriptors grouped by size (classes are contiguous ranges)
    std::vector<int> order(B);
    for (int q = 0; q < B; ++q) order[q] = q;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b->n[x] < b->n[y]; });
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
    struct Cls { int first, count, n; };
    std::vector<Cls> classes;
    for (int k = 0; k < B;) {
        int e = k;
        while (e < B && desc[e].n == desc[k].n) ++e;
        classes.push_back({k, e - k, desc[k].n});
        k = e;
    }
    TrainLayer layers[4];
    int64_t woff = 0;
    for (int l = 0; l < 4; ++l) {
        layers[l].cin = net->ch[l];
        layers[l].cout = net->ch[l + 1];
        layers[l].woff = woff;
        layers[l].boff = woff + (int64_t)layers[l].cout * layers[l].cin * 9;
        woff = layers[l].boff + layers[l].cout;
    }
    TrainProb *d_desc = (TrainProb *)(base + off_desc);
    float *wpart = (float *)(base + off_wpart);
    float *loss_part = (float *)(base + off_loss);
    float *d_loss = loss_part + B * J;

    MG_TRY(net->join.enter());
    hipStream_t st = net->join.internal;
    // the upload's source must outlive the asynchronous copy: keep the bytes in the network object
    net->host_desc.assign((const char *)desc.data(), (const char *)(desc.data() + B));
    MG_HIP(hipMemcpyAsync(d_desc, net->host_desc.data(), sizeof(TrainProb) * B, hipMemcpyHostToDevice, st));
    const float scale = 1.0f / ((float)B * (float)J);
    for (const Cls &c : classes) launch_tr_input(d_desc + c.first, c.count, c.n, st);
    for (int l = 0; l < 4; ++l)
        for (const Cls &c : classes) launch_tr_conv_fwd(d_desc + c.first, c.count, c.n, net->params, layers[l], l, st);
    for (const Cls &c : classes) {
        launch_tr_av(d_desc + c.first, c.count, c.n, J, st);
        launch_tr_residual_norm(d_desc + c.first, c.count, J, (float)o.omega, loss_part, st);
        launch_tr_dout(d_desc + c.first, c.count, c.n, J, scale, st);
    }
    for (int l = 3; l >= 0; --l) {
        for (const Cls &c : classes) {
            launch_tr_conv_bwd_weight(d_desc + c.first, c.count, layers[l], l, wpart, net->np, st);
            if (l > 0) launch_tr_conv_bwd_data(d_desc + c.first, c.count, c.n, net->params, layers[l], l, st);
        }
    }
    launch_tr_reduce(wpart, B, net->np, net->grad, st);
    launch_tr_loss(loss_part, B * J, scale, d_loss, st);
    if (o.apply_update) {
        net->step += 1;
        const double t = (double)net->step;
        const float c1 = (float)(1.0 - std::pow((double)o.beta1, t));
        const float c2 = (float)(1.0 - std::pow((double)o.beta2, t));
        launch_adam(net->np, net->params, net->m, net->v, net->grad, o.lr, o.beta1, o.beta2, o.adam_eps, c1, c2, st);
        net->packed_valid = false;
    }
    MG_HIP(hipGetLastError());
    if (loss || grad) {
        if (loss) MG_HIP(hipMemcpyAsync(loss, d_loss, sizeof(float), hipMemcpyDeviceToHost, st));
        if (grad) MG_HIP(hipMemcpyAsync(grad, net->grad, sizeof(float) * net->np, hipMemcpyDeviceToHost, st));
        MG_HIP(hipStreamSynchronize(st));
    }
    return net->join.leave();
}
