// Smoother network objects: parameters (FP32 master copy on the device), Adam
// state, checkpoints, and the training step driver.
#include <cstdio>
#include <cstring>
#include <vector>

#include "internal.hpp"
#include "launch.hpp"

using namespace mg;

namespace {

constexpr uint32_t kMagic = 0x4e4e434d;  // "MCNN"
constexpr uint32_t kVersion = 1;

int64_t count_params(int nl, const int *ch)
{
    int64_t np = 0;
    for (int l = 0; l < nl; ++l) np += (int64_t)ch[l + 1] * ch[l] * 9 + ch[l + 1];
    return np;
}

mg_status check_net(mg_net net)
{
    if (!net) return set_error(MG_ERR_ARG, "net is null");
    return MG_OK;
}

}  // namespace

namespace mg {

mg_status net_params64(mg_net net, hipStream_t st)
{
    launch_f32_to_f64(net->np, net->params, net->params64, st);
    MG_HIP(hipGetLastError());
    return MG_OK;
}

mg_status net_pack_mfma(mg_net net, hipStream_t st)
{
    if (net->packed_valid) return MG_OK;
    launch_pack_weights_mfma(net->params, net->packed, st);
    MG_HIP(hipGetLastError());
    net->packed_valid = true;
    return MG_OK;
}

}  // namespace mg

extern "C" {

mg_status mg_net_create(const mg_net_desc *d, void *stream, mg_net *out)
{
    clear_error();
    if (!out) return set_error(MG_ERR_ARG, "out is null");
    *out = nullptr;
    static const int want[5] = {9, 32, 32, 32, 25};
    if (d) {
        if (d->nlayers != 4 || !d->channels) return set_error(MG_ERR_ARG, "the network must have 4 layers");
        for (int l = 0; l < 5; ++l)
            if (d->channels[l] != want[l]) return set_error(MG_ERR_ARG, "channels must be {9, 32, 32, 32, 25}");
    }
    MG_TRY(require_device());
    mg_net net = new mg_net_s();
    net->np = count_params(4, want);
    mg_status s = net->join.init((hipStream_t)stream);
    net->arena.stream = net->scratch.stream = net->join.internal;
    if (s == MG_OK) s = net->arena.alloc((void **)&net->params, net->np * sizeof(float));
    if (s == MG_OK) s = net->arena.alloc((void **)&net->m, net->np * sizeof(float));
    if (s == MG_OK) s = net->arena.alloc((void **)&net->v, net->np * sizeof(float));
    if (s == MG_OK) s = net->arena.alloc((void **)&net->grad, net->np * sizeof(float));
    if (s == MG_OK) s = net->arena.alloc((void **)&net->params64, net->np * sizeof(double));
    if (s == MG_OK) s = net->arena.alloc(&net->packed, packed_net_bytes());
    if (s < 0) {
        net->arena.release();
        net->join.destroy();
        delete net;
        return s;
    }
    *out = net;
    return MG_OK;
}

mg_status mg_net_destroy(mg_net net)
{
    clear_error();
    if (!net) return MG_OK;
    if (net->join.internal) (void)hipStreamSynchronize(net->join.internal);
    train_draw_release(*net);
    net->scratch.release();
    net->arena.release();
    net->join.destroy();
    delete net;
    return MG_OK;
}

mg_status mg_net_num_params(mg_net net, int64_t *np)
{
    clear_error();
    MG_TRY(check_net(net));
    if (!np) return set_error(MG_ERR_ARG, "np is null");
    *np = net->np;
    return MG_OK;
}

mg_status mg_net_get(mg_net net, float *host, int64_t len)
{
    clear_error();
    MG_TRY(check_net(net));
    if (!host || len != net->np) return set_error(MG_ERR_SHAPE, "need a host buffer of %lld floats", (long long)net->np);
    MG_TRY(net->join.enter());
    MG_HIP(hipMemcpyAsync(host, net->params, net->np * sizeof(float), hipMemcpyDeviceToHost, net->join.internal));
    MG_HIP(hipStreamSynchronize(net->join.internal));
    return net->join.leave();
}

mg_status mg_net_set(mg_net net, const float *host, int64_t len)
{
    clear_error();
    MG_TRY(check_net(net));
    if (!host || len != net->np) return set_error(MG_ERR_SHAPE, "need a host buffer of %lld floats", (long long)net->np);
    MG_TRY(net->join.enter());
    hipStream_t st = net->join.internal;
    MG_HIP(hipMemcpyAsync(net->params, host, net->np * sizeof(float), hipMemcpyHostToDevice, st));
    MG_HIP(hipMemsetAsync(net->m, 0, net->np * sizeof(float), st));
    MG_HIP(hipMemsetAsync(net->v, 0, net->np * sizeof(float), st));
    MG_HIP(hipStreamSynchronize(st));
    net->step = 0;
    net->packed_valid = false;
    return net->join.leave();
}

mg_status mg_net_save(mg_net net, const char *path)
{
    clear_error();
    MG_TRY(check_net(net));
    if (!path) return set_error(MG_ERR_ARG, "path is null");
    std::vector<float> buf(3 * net->np);
    MG_TRY(net->join.enter());
    hipStream_t st = net->join.internal;
    MG_HIP(hipMemcpyAsync(buf.data(), net->params, net->np * sizeof(float), hipMemcpyDeviceToHost, st));
    MG_HIP(hipMemcpyAsync(buf.data() + net->np, net->m, net->np * sizeof(float), hipMemcpyDeviceToHost, st));
    MG_HIP(hipMemcpyAsync(buf.data() + 2 * net->np, net->v, net->np * sizeof(float), hipMemcpyDeviceToHost, st));
    MG_HIP(hipStreamSynchronize(st));
    FILE *fp = std::fopen(path, "wb");
    if (!fp) return set_error(MG_ERR_ARG, "cannot open %s for writing", path);
    const uint32_t hdr[4] = {kMagic, kVersion, 4u, 0u};
    const int32_t ch[5] = {9, 32, 32, 32, 25};
    const int64_t meta[2] = {net->np, net->step};
    bool ok = std::fwrite(hdr, sizeof hdr, 1, fp) == 1 && std::fwrite(ch, sizeof ch, 1, fp) == 1 &&
              std::fwrite(meta, sizeof meta, 1, fp) == 1 &&
              std::fwrite(buf.data(), sizeof(float), buf.size(), fp) == buf.size();
    ok = (std::fclose(fp) == 0) && ok;
    if (!ok) return set_error(MG_ERR_ARG, "write to %s failed", path);
    return net->join.leave();
}

mg_status mg_net_load(mg_net net, const char *path)
{
    clear_error();
    MG_TRY(check_net(net));
    if (!path) return set_error(MG_ERR_ARG, "path is null");
    FILE *fp = std::fopen(path, "rb");
    if (!fp) return set_error(MG_ERR_ARG, "cannot open %s", path);
    uint32_t hdr[4];
    int32_t ch[5];
    int64_t meta[2];
    std::vector<float> buf(3 * net->np);
    bool ok = std::fread(hdr, sizeof hdr, 1, fp) == 1 && std::fread(ch, sizeof ch, 1, fp) == 1 &&
              std::fread(meta, sizeof meta, 1, fp) == 1;
    ok = ok && hdr[0] == kMagic && hdr[1] == kVersion && hdr[2] == 4u && meta[0] == net->np;
    ok = ok && ch[0] == 9 && ch[1] == 32 && ch[2] == 32 && ch[3] == 32 && ch[4] == 25;
    ok = ok && std::fread(buf.data(), sizeof(float), buf.size(), fp) == buf.size();
    std::fclose(fp);
    if (!ok) return set_error(MG_ERR_ARG, "%s is not a compatible checkpoint", path);
    MG_TRY(net->join.enter());
    hipStream_t st = net->join.internal;
    MG_HIP(hipMemcpyAsync(net->params, buf.data(), net->np * sizeof(float), hipMemcpyHostToDevice, st));
    MG_HIP(hipMemcpyAsync(net->m, buf.data() + net->np, net->np * sizeof(float), hipMemcpyHostToDevice, st));
    MG_HIP(hipMemcpyAsync(net->v, buf.data() + 2 * net->np, net->np * sizeof(float), hipMemcpyHostToDevice, st));
    MG_HIP(hipStreamSynchronize(st));
    net->step = meta[1];
    net->packed_valid = false;
    return net->join.leave();
}

}  // extern "C"

// Training step: see train.cpp.
