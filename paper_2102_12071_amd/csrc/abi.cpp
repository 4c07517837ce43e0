// C ABI plumbing: error state, status strings, defaults, device checks,
// allocation arenas, stream joins, and the stand-alone discretisation calls.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "internal.hpp"
#include "launch.hpp"

namespace mg {

namespace {
thread_local std::string g_error;
}

mg_status set_error(mg_status s, const char *fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return s;
}

void clear_error() { g_error.clear(); }

mg_status require_device()
{
    static int checked = 0;  // 1 ok, -1 wrong device
    static std::string why;
    if (checked == 1) return MG_OK;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(MG_ERR_DEVICE, "no HIP device: %s", hipGetErrorString(e));
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return set_error(MG_ERR_DEVICE, "hipGetDeviceProperties: %s", hipGetErrorString(e));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return set_error(MG_ERR_DEVICE, "this library is built for gfx950 (MI355X); device %d is %s", dev,
                         prop.gcnArchName);
    checked = 1;
    return MG_OK;
}

// Sub-allocates 256-byte aligned, zeroed pieces from chunks of at least
// kArenaChunk bytes (one hipMalloc and one memset per chunk).
mg_status Arena::alloc(void **p, size_t bytes)
{
    constexpr size_t kArenaChunk = (size_t)64 << 20;
    *p = nullptr;
    bytes = (bytes + 255) & ~(size_t)255;
    if (bytes == 0) bytes = 256;
    if (blocks.empty() || used + bytes > cap) {
        const size_t want = bytes > kArenaChunk ? bytes : kArenaChunk;
        void *q = nullptr;
        hipError_t e = hipMalloc(&q, want);
        if (e != hipSuccess) {
            return set_error(e == hipErrorOutOfMemory ? MG_ERR_OOM : MG_ERR_DEVICE, "hipMalloc(%zu): %s", want,
                             hipGetErrorString(e));
        }
        blocks.push_back(q);
        e = hipMemsetAsync(q, 0, want, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return set_error(MG_ERR_DEVICE, "clearing a new chunk: %s", hipGetErrorString(e));
        cap = want;
        used = 0;
    }
    *p = (char *)blocks.back() + used;
    used += bytes;
    return MG_OK;
}

void Arena::release()
{
    for (void *q : blocks) (void)hipFree(q);
    blocks.clear();
    cap = used = 0;
}

mg_status StreamJoin::init(hipStream_t user_stream)
{
    user = user_stream;
    MG_HIP(hipStreamCreateWithFlags(&internal, hipStreamNonBlocking));
    MG_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    return MG_OK;
}

mg_status StreamJoin::enter()
{
    MG_HIP(hipEventRecord(ev, user));
    MG_HIP(hipStreamWaitEvent(internal, ev, 0));
    return MG_OK;
}

mg_status StreamJoin::leave()
{
    MG_HIP(hipEventRecord(ev, internal));
    MG_HIP(hipStreamWaitEvent(user, ev, 0));
    return MG_OK;
}

void StreamJoin::destroy()
{
    if (internal) {
        (void)hipStreamSynchronize(internal);
        (void)hipStreamDestroy(internal);
    }
    if (ev) (void)hipEventDestroy(ev);
    internal = nullptr;
    ev = nullptr;
}

}  // namespace mg

using namespace mg;

namespace {
bool odd_in_range(int n, int lo, int hi) { return n >= lo && n <= hi && (n & 1) == 1; }
}  // namespace

extern "C" {

const char *mg_status_str(mg_status s)
{
    switch (s) {
    case MG_OK: return "MG_OK";
    case MG_NOT_CONVERGED: return "MG_NOT_CONVERGED";
    case MG_ERR_ARG: return "MG_ERR_ARG";
    case MG_ERR_SHAPE: return "MG_ERR_SHAPE";
    case MG_ERR_DEVICE: return "MG_ERR_DEVICE";
    case MG_ERR_DIVERGED: return "MG_ERR_DIVERGED";
    case MG_ERR_STATE: return "MG_ERR_STATE";
    case MG_ERR_OOM: return "MG_ERR_OOM";
    }
    return "MG_UNKNOWN_STATUS";
}

const char *mg_last_error(void) { return mg::g_error.c_str(); }

const char *mg_version(void) { return "mgcnn 0.1.0 (gfx950)"; }

void mg_options_default(mg_options *opt)
{
    if (!opt) return;
    std::memset(opt, 0, sizeof *opt);
    opt->smoother = MG_SMOOTHER_JACOBI;
    opt->nu_pre = 1;
    opt->nu_post = 1;
    opt->omega = 2.0 / 3.0;
    opt->coarsest_n = 7;
    opt->precision = MG_PREC_MIXED;
    opt->use_graph = 1;
    opt->check_every = 16;
    opt->fallback = 0;
}

void mg_train_opts_default(mg_train_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->lr = 1e-3f;
    o->beta1 = 0.9f;
    o->beta2 = 0.999f;
    o->adam_eps = 1e-8f;
    o->omega = 2.0 / 3.0;
    o->precision = 1;
    o->apply_update = 1;
}

mg_status mg_stencil_q1_rotated(int32_t n, double theta, double eps, double *out, void *stream)
{
    clear_error();
    if (!odd_in_range(n, 1, 16383)) return set_error(MG_ERR_ARG, "n must be odd in [1, 16383], got %d", n);
    if (!out) return set_error(MG_ERR_ARG, "out is null");
    if (!(eps > 0.0 && eps <= 1.0) || !std::isfinite(theta))
        return set_error(MG_ERR_ARG, "need 0 < eps <= 1 and finite theta");
    MG_TRY(require_device());
    launch_q1_rotated(n, n, (int64_t)n * n, theta, eps, out, (hipStream_t)stream);
    MG_HIP(hipGetLastError());
    return MG_OK;
}

mg_status mg_stencil_cellavg5(int32_t n, const double *a, double *out, void *stream)
{
    clear_error();
    if (!odd_in_range(n, 1, 16383)) return set_error(MG_ERR_ARG, "n must be odd in [1, 16383], got %d", n);
    if (!a || !out) return set_error(MG_ERR_ARG, "null pointer");
    MG_TRY(require_device());
    launch_cellavg5(n, a, n + 1, n, (int64_t)n * n, out, (hipStream_t)stream);
    MG_HIP(hipGetLastError());
    return MG_OK;
}

mg_status mg_galerkin(int32_t n, const double *A, double *Ac, void *stream)
{
    clear_error();
    if (!odd_in_range(n, 3, 16383)) return set_error(MG_ERR_ARG, "n must be odd in [3, 16383], got %d", n);
    if (!A || !Ac) return set_error(MG_ERR_ARG, "null pointer");
    MG_TRY(require_device());
    const int nc = (n - 1) / 2;
    launch_galerkin(n, n, (int64_t)n * n, A, nc, (int64_t)nc * nc, Ac, (hipStream_t)stream);
    MG_HIP(hipGetLastError());
    return MG_OK;
}

mg_status mg_stencil_mask(int32_t n, const uint8_t *mask, const double *A, double *out, void *stream)
{
    clear_error();
    if (!odd_in_range(n, 1, 16383)) return set_error(MG_ERR_ARG, "n must be odd in [1, 16383], got %d", n);
    if (!mask || !A || !out) return set_error(MG_ERR_ARG, "null pointer");
    MG_TRY(require_device());
    launch_mask(n, mask, A, out, (hipStream_t)stream);
    MG_HIP(hipGetLastError());
    return MG_OK;
}

}  // extern "C"
