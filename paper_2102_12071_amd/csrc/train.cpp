// Training step driver for the high-frequency smoothing loss: groups the
// batch by grid size and runs forward, loss, backward and Adam on the device,
// either in FP32 on the vector units (precision 0, the parity path) or in
// BF16 on the matrix cores with FP32 accumulation (precision 1).
#include <algorithm>
#include <cmath>
#include <cstring>
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
// instead of coming from the high-frequency loss.  prepare uploads the
// problem table (before a graph capture, never inside one); enqueue only
// launches kernels.
struct Fp32Plan {
    char *base = nullptr;  // the step's scratch
    std::vector<int> order;
    std::vector<Cls> classes;
    TrainProb *d_desc = nullptr;
    float *wpart = nullptr;
    TrainLayer layers[4];
};

mg_status prepare_fp32(mg_net_s &net, const mg_train_batch *b, Fp32Plan &pl, hipStream_t st)
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
    char *base = pl.base;
    classes_of(b, pl.order, pl.classes);
    std::vector<TrainProb> desc(B);
    for (int k = 0; k < B; ++k) {
        const int q = pl.order[k];
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
    layer_offsets(net, pl.layers);
    pl.d_desc = (TrainProb *)(base + off_desc);
    pl.wpart = (float *)(base + off_wpart);
    return upload_desc(net, desc, pl.d_desc, st);
}

void enqueue_fp32(mg_net_s &net, const mg_train_batch *b, const mg_train_opts &o, const Fp32Plan &pl,
                  float *loss_part, hipStream_t st, bool ext = false)
{
    const int B = b->nprob, J = b->nvec;
    const TrainProb *d_desc = pl.d_desc;
    const float scale = J > 0 ? 1.0f / ((float)B * (float)J) : 0.0f;
    for (const Cls &c : pl.classes) launch_tr_input(d_desc + c.first, c.count, c.n, st);
    for (int l = 0; l < 4; ++l)
        for (const Cls &c : pl.classes)
            launch_tr_conv_fwd(d_desc + c.first, c.count, c.n, net.params, pl.layers[l], l, st);
    for (const Cls &c : pl.classes) {
        if (ext) {
            launch_tr_dout_ext(d_desc + c.first, c.count, c.n, st);
            continue;
        }
        launch_tr_av(d_desc + c.first, c.count, c.n, J, st);
        launch_tr_residual_norm(d_desc + c.first, c.count, J, (float)o.omega, loss_part, st);
        launch_tr_dout(d_desc + c.first, c.count, c.n, J, scale, st);
    }
    for (int l = 3; l >= 0; --l) {
        for (const Cls &c : pl.classes) {
            launch_tr_conv_bwd_weight(d_desc + c.first, c.count, pl.layers[l], l, pl.wpart, net.np, st);
            if (l > 0) launch_tr_conv_bwd_data(d_desc + c.first, c.count, c.n, net.params, pl.layers[l], l, st);
        }
    }
    launch_tr_reduce(pl.wpart, B, net.np, net.grad, st);
}

mg_status step_fp32(mg_net_s &net, const mg_train_batch *b, const mg_train_opts &o, float *loss_part,
                    hipStream_t st, bool ext = false)
{
    Fp32Plan pl;
    pl.base = (char *)net.scratch_base;
    MG_TRY(prepare_fp32(net, b, pl, st));
    enqueue_fp32(net, b, o, pl, loss_part, st, ext);
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
    int ntiles, resblk;  // ntiles: weight-gradient parts (tile groups)
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
        L.ntiles += trb_tile_groups(b->n[q]);
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

struct Bf16Plan {
    char *base = nullptr;  // the step's scratch
    std::vector<int> order;
    std::vector<Cls> classes;
    TrainProbB *d_desc = nullptr;
    float *part = nullptr;
    bf16_t *pf[4], *pb[4];
    float *bias[4];
    TrainLayer layers[4];
};

mg_status prepare_bf16(mg_net_s &net, const mg_train_batch *b, const Bf16Layout &L, Bf16Plan &pl, hipStream_t st)
{
    const int B = b->nprob, J = b->nvec;
    char *base = pl.base;
    classes_of(b, pl.order, pl.classes);
    std::vector<TrainProbB> desc(B);
    int part0 = 0;
    for (int k = 0; k < B; ++k) {
        const int q = pl.order[k];
        const int n = b->n[q];
        const int64_t v = (int64_t)n * n;
        char *p = base + L.off[q];
        TrainProbB &d = desc[k];
        d.index = q;
        d.n = n;
        d.plane = v;
        d.part0 = part0;
        part0 += trb_tile_groups(n);
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
    layer_offsets(net, pl.layers);
    pl.d_desc = (TrainProbB *)(base + L.desc);
    pl.part = (float *)(base + L.part);
    for (int l = 0; l < 4; ++l) {
        pl.pf[l] = (bf16_t *)(base + L.pack_fwd[l]);
        pl.pb[l] = (bf16_t *)(base + L.pack_bwd[l]);
        pl.bias[l] = (float *)(base + L.bias[l]);
    }
    return upload_desc(net, desc, pl.d_desc, st);
}

void enqueue_bf16(mg_net_s &net, const mg_train_batch *b, const mg_train_opts &o, const Bf16Layout &L,
                  const Bf16Plan &pl, float *loss_part, hipStream_t st)
{
    const int B = b->nprob, J = b->nvec;
    char *base = pl.base;
    const TrainProbB *d_desc = pl.d_desc;
    TrbPackJobs jobs;
    for (int l = 0; l < 4; ++l) {
        jobs.layer[l] = pl.layers[l];
        jobs.fwd[l] = pl.pf[l];
        jobs.bwd[l] = pl.pb[l];
        jobs.bias[l] = pl.bias[l];
    }
    launch_trb_pack_all(net.params, jobs, st);
    const float scale = 1.0f / ((float)B * (float)J);
    for (const Cls &c : pl.classes) launch_trb_input(d_desc + c.first, c.count, c.n, st);
    for (int l = 0; l < 4; ++l)
        for (const Cls &c : pl.classes)
            launch_trb_conv_fwd(d_desc + c.first, c.count, c.n, l, pl.pf[l], pl.bias[l], st);
    for (const Cls &c : pl.classes) {
        launch_trb_av(d_desc + c.first, c.count, c.n, J, st);
        launch_trb_residual_norm(d_desc + c.first, c.count, c.n, J, (float)o.omega, loss_part,
                                 (double *)(base + L.respart), L.resblk, st);
        launch_trb_dout(d_desc + c.first, c.count, c.n, J, scale, st);
    }
    for (int l = 3; l >= 0; --l) {
        const TrainLayer &ly = pl.layers[l];
        for (const Cls &c : pl.classes) launch_trb_wgrad(d_desc + c.first, c.count, c.n, l, ly.cout, pl.part, st);
        launch_trb_reduce(pl.part, L.ntiles, ly.cin, ly.cout, ly.woff, ly.boff, net.grad, (float *)(base + L.part2),
                          st);
        if (l > 0)
            for (const Cls &c : pl.classes) launch_trb_conv_bwd_data(d_desc + c.first, c.count, c.n, l, pl.pb[l], st);
    }
}

mg_status step_bf16(mg_net_s &net, const mg_train_batch *b, const mg_train_opts &o, const Bf16Layout &L,
                    float *loss_part, hipStream_t st)
{
    Bf16Plan pl;
    pl.base = (char *)net.scratch_base;
    MG_TRY(prepare_bf16(net, b, L, pl, st));
    enqueue_bf16(net, b, o, L, pl, loss_part, st);
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
    return step_fp32(net, &b, o, nullptr, st, true);
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

// ---------------------------------------------------------------------------
// Training steps on drawn problems, replayed from one captured HIP graph.
// The graph holds every launch of a step: the problems' stencils from their
// tensors, the gather of their high-frequency vectors from the pools, forward,
// loss, backward and Adam (its bias corrections from a device step count).
// What changes from step to step - the tensors, the pool indices, the step
// count - lives in a small device block written before each replay from a
// pinned staging copy; the problem sizes, pools and options fix the graph, and
// a step whose structure differs rebuilds it.
namespace mg {

struct TrainDraw {
    // structure of the captured step
    std::vector<int> n, pool_n, pool_size;
    std::vector<const float *> pools;
    int J = 0, precision = -1, apply = -1;
    float lr = 0, b1 = 0, b2 = 0, eps = 0;
    double omega = 0;
    // problems in size order: slot k holds problem order[k]
    std::vector<int> order, slot_of;
    std::vector<Cls> classes;
    std::vector<const float *> class_pool;
    Arena arena;            // buffers and scratch of this structure
    double *stencils = nullptr;
    float *vectors = nullptr;
    char *dev_stage = nullptr;   // k [B][3] doubles, t (int64), index [B][J] ints
    char *host_stage = nullptr;  // pinned
    size_t stage_bytes = 0, off_t = 0, off_index = 0;
    float *loss_part = nullptr, *d_loss = nullptr;
    hipEvent_t staged = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<const double *> sptr;
    std::vector<const float *> vptr;

    void release()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (staged) (void)hipEventDestroy(staged);
        if (host_stage) (void)hipHostFree(host_stage);
        exec = nullptr;
        graph = nullptr;
        staged = nullptr;
        host_stage = nullptr;
        arena.release();
    }
};

void train_draw_release(mg_net_s &net)
{
    if (net.draw) {
        net.draw->release();
        delete net.draw;
        net.draw = nullptr;
    }
}

}  // namespace mg

namespace {

bool same_structure(const TrainDraw &t, const mg_train_draw *d, const mg_train_opts &o)
{
    if (t.precision != o.precision || t.apply != o.apply_update || t.J != d->nvec || (int)t.n.size() != d->nprob ||
        (int)t.pools.size() != d->npools || t.lr != o.lr || t.b1 != o.beta1 || t.b2 != o.beta2 ||
        t.eps != o.adam_eps || t.omega != o.omega)
        return false;
    for (int q = 0; q < d->nprob; ++q)
        if (t.n[q] != d->n[q]) return false;
    for (int p = 0; p < d->npools; ++p)
        if (t.pools[p] != d->pool[p] || t.pool_n[p] != d->pool_n[p] || t.pool_size[p] != d->pool_size[p]) return false;
    return true;
}

mg_status build_draw(mg_net_s &net, const mg_train_draw *d, const mg_train_opts &o, hipStream_t st)
{
    MG_HIP(hipStreamSynchronize(st));
    train_draw_release(net);
    net.draw = new TrainDraw();
    TrainDraw &t = *net.draw;
    const int B = d->nprob, J = d->nvec;
    t.arena.stream = st;
    t.n.assign(d->n, d->n + B);
    t.pools.assign(d->pool, d->pool + d->npools);
    t.pool_n.assign(d->pool_n, d->pool_n + d->npools);
    t.pool_size.assign(d->pool_size, d->pool_size + d->npools);
    t.J = J;
    t.precision = o.precision;
    t.apply = o.apply_update;
    t.lr = o.lr;
    t.b1 = o.beta1;
    t.b2 = o.beta2;
    t.eps = o.adam_eps;
    t.omega = o.omega;
    // size order (stable), the buffers of slot k at running offsets
    t.order.resize(B);
    for (int q = 0; q < B; ++q) t.order[q] = q;
    std::stable_sort(t.order.begin(), t.order.end(), [&](int x, int y) { return d->n[x] < d->n[y]; });
    t.slot_of.resize(B);
    for (int k = 0; k < B; ++k) t.slot_of[t.order[k]] = k;
    size_t sten = 0, vec = 0;
    std::vector<size_t> soff(B), voff(B);
    for (int k = 0; k < B; ++k) {
        const size_t nn = (size_t)d->n[t.order[k]] * d->n[t.order[k]];
        soff[k] = sten;
        voff[k] = vec;
        sten += 9 * nn;
        vec += (size_t)J * nn;
    }
    void *p = nullptr;
    MG_TRY(t.arena.alloc(&p, sten * sizeof(double)));
    t.stencils = (double *)p;
    MG_TRY(t.arena.alloc(&p, vec * sizeof(float)));
    t.vectors = (float *)p;
    t.off_t = (size_t)B * 3 * sizeof(double);
    t.off_index = t.off_t + sizeof(int64_t);
    t.stage_bytes = t.off_index + (size_t)B * J * sizeof(int);
    MG_TRY(t.arena.alloc(&p, t.stage_bytes));
    t.dev_stage = (char *)p;
    MG_HIP(hipHostMalloc((void **)&t.host_stage, t.stage_bytes, hipHostMallocDefault));
    MG_HIP(hipEventCreateWithFlags(&t.staged, hipEventDisableTiming));
    t.sptr.resize(B);
    t.vptr.resize(B);
    for (int q = 0; q < B; ++q) {
        const int k = t.slot_of[q];
        t.sptr[q] = t.stencils + soff[k];
        t.vptr[q] = t.vectors + voff[k];
    }
    t.classes.clear();
    t.class_pool.clear();
    for (int k = 0; k < B;) {
        int e = k;
        while (e < B && d->n[t.order[e]] == d->n[t.order[k]]) ++e;
        const int n = d->n[t.order[k]];
        t.classes.push_back({k, e - k, n});
        const float *pool = nullptr;
        for (int q = 0; q < d->npools; ++q)
            if (d->pool_n[q] == n) pool = d->pool[q];
        t.class_pool.push_back(pool);
        k = e;
    }
    // the step's scratch and problem table, then the capture
    const mg_train_batch b{B, t.n.data(), t.sptr.data(), t.vptr.data(), J};
    Bf16Layout L16;
    Bf16Plan p16;
    Fp32Plan p32;
    size_t need = o.precision == 1 ? (L16 = bf16_layout(&b)).bytes : fp32_scratch(net, &b);
    const size_t loss_bytes = ((sizeof(float) * (B * J + 1)) + 255) & ~(size_t)255;
    MG_TRY(t.arena.alloc(&p, need + loss_bytes));
    t.loss_part = (float *)((char *)p + need);
    t.d_loss = t.loss_part + B * J;
    if (o.precision == 1) {
        p16.base = (char *)p;
        MG_TRY(prepare_bf16(net, &b, L16, p16, st));
    } else {
        p32.base = (char *)p;
        MG_TRY(prepare_fp32(net, &b, p32, st));
    }
    MG_HIP(hipStreamSynchronize(st));
    const double *dk = (const double *)t.dev_stage;
    const int64_t *dt = (const int64_t *)(t.dev_stage + t.off_t);
    const int *didx = (const int *)(t.dev_stage + t.off_index);
    MG_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    for (size_t c = 0; c < t.classes.size(); ++c) {
        const Cls &cl = t.classes[c];
        const size_t nn = (size_t)cl.n * cl.n;
        double *sdst = t.stencils + soff[cl.first];
        float *vdst = t.vectors + voff[cl.first];
        launch_q1_rotated_batch(cl.n, cl.count, dk + 3 * cl.first, sdst, st);
        launch_tr_gather(cl.n, cl.count, J, t.class_pool[c], didx + (size_t)cl.first * J, vdst, st);
        (void)nn;
    }
    if (o.precision == 1)
        enqueue_bf16(net, &b, o, L16, p16, t.loss_part, st);
    else
        enqueue_fp32(net, &b, o, p32, t.loss_part, st);
    launch_tr_loss(t.loss_part, B * J, 1.0f / ((float)B * (float)J), t.d_loss, st);
    if (o.apply_update) launch_adam_dev(net.np, net.params, net.m, net.v, net.grad, o.lr, o.beta1, o.beta2, o.adam_eps,
                                        dt, st);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &g);
    if (e != hipSuccess) return set_error(MG_ERR_DEVICE, "training graph capture failed: %s", hipGetErrorString(e));
    t.graph = g;
    MG_HIP(hipGraphInstantiate(&t.exec, t.graph, nullptr, nullptr, 0));
    return MG_OK;
}

}  // namespace

extern "C" mg_status mg_train_step_draw(mg_net net, const mg_train_draw *d, const mg_train_opts *o_in, float *loss,
                                        float *grad)
{
    clear_error();
    if (!net) return set_error(MG_ERR_ARG, "net is null");
    if (!d || d->nprob < 1 || !d->n || !d->theta || !d->eps || d->nvec < 1 || d->npools < 1 || !d->pool_n ||
        !d->pool || !d->pool_size || !d->index)
        return set_error(MG_ERR_ARG, "a drawn batch needs nprob >= 1, sizes, tensors, pools, indices and nvec >= 1");
    mg_train_opts o;
    if (o_in)
        o = *o_in;
    else
        mg_train_opts_default(&o);
    MG_TRY(check_train_opts(o));
    const int B = d->nprob, J = d->nvec;
    if ((int64_t)B * J > (1 << 26)) return set_error(MG_ERR_ARG, "nprob * nvec too large");
    for (int q = 0; q < B; ++q) {
        const int n = d->n[q];
        if (n < 3 || n > 255 || (n & 1) == 0) return set_error(MG_ERR_ARG, "problem %d: n = %d must be odd in [3, 255]", q, n);
        if (!(d->eps[q] > 0.0 && d->eps[q] <= 1.0) || !std::isfinite(d->theta[q]))
            return set_error(MG_ERR_ARG, "problem %d: need 0 < eps <= 1 and finite theta", q);
        int pool = -1;
        for (int p = 0; p < d->npools; ++p)
            if (d->pool_n[p] == n) pool = p;
        if (pool < 0 || !d->pool[pool] || d->pool_size[pool] < 1)
            return set_error(MG_ERR_ARG, "problem %d: no vector pool of size %d", q, n);
        for (int j = 0; j < J; ++j) {
            const int ix = d->index[(size_t)q * J + j];
            if (ix < 0 || ix >= d->pool_size[pool])
                return set_error(MG_ERR_ARG, "problem %d: pool index %d out of [0, %d)", q, ix, d->pool_size[pool]);
        }
    }
    MG_TRY(net->join.enter());
    hipStream_t st = net->join.internal;
    if (!net->draw || !same_structure(*net->draw, d, o)) MG_TRY(build_draw(*net, d, o, st));
    TrainDraw &t = *net->draw;
    // the previous step's upload must have left the staging block
    MG_HIP(hipEventSynchronize(t.staged));
    double *hk = (double *)t.host_stage;
    int *hidx = (int *)(t.host_stage + t.off_index);
    for (int q = 0; q < B; ++q) {
        const int k = t.slot_of[q];
        q1_tensor(d->theta[q], d->eps[q], hk + 3 * k);
        std::memcpy(hidx + (size_t)k * J, d->index + (size_t)q * J, sizeof(int) * J);
    }
    const int64_t tnext = net->step + 1;
    std::memcpy(t.host_stage + t.off_t, &tnext, sizeof tnext);
    MG_HIP(hipMemcpyAsync(t.dev_stage, t.host_stage, t.stage_bytes, hipMemcpyHostToDevice, st));
    MG_HIP(hipEventRecord(t.staged, st));
    MG_HIP(hipGraphLaunch(t.exec, st));
    if (o.apply_update) {
        net->step = tnext;
        net->packed_valid = false;
    }
    MG_HIP(hipGetLastError());
    if (loss || grad) {
        if (loss) MG_HIP(hipMemcpyAsync(loss, t.d_loss, sizeof(float), hipMemcpyDeviceToHost, st));
        if (grad) MG_HIP(hipMemcpyAsync(grad, net->grad, sizeof(float) * net->np, hipMemcpyDeviceToHost, st));
        MG_HIP(hipStreamSynchronize(st));
    }
    return net->join.leave();
}

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
        MG_TRY(step_fp32(*net, b, o, loss_part, st));
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
