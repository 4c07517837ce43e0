// Flexible GMRES with the multigrid cycle as the preconditioner (section 6,
// "incorporation with FGMRES"): restarted FGMRES(m) of Saad, right-
// preconditioned, one V-cycle of the context per iteration.  The cycle is
// mixed precision (or FP64) and so not exactly a fixed linear operator; the
// flexible variant keeps every preconditioned direction z_j and builds the
// update from them, which stays correct for a preconditioner that varies.
//
// Problems of a context are solved one after another; the cycle is launched
// for the current problem only (the context's compacted launches).  Every
// vector is FP64 on the problem's finest grid.  Orthogonalisation is
// classical Gram-Schmidt applied twice, so that an iteration needs one
// round trip to the host (the Hessenberg column, the Givens rotations and the
// residual estimate are computed there); the rest runs on the library stream.
#include <cmath>
#include <vector>

#include "internal.hpp"
#include "launch.hpp"

using namespace mg;

namespace {

// Where an FGMRES(m) solve keeps its vectors: 2 m + 4 FP64 vectors of vs values (V: m + 1, Z: m,
// w, X, r) and the small arrays (partial sums of m + 2 dot products, two Hessenberg columns, the
// coefficients, a norm).  restart: the m the layout was made for (>= the solve's m).
struct Workspace {
    double *vec = nullptr, *small = nullptr;
    int restart = 0;
    int64_t vs = 0;
};

int64_t vector_stride(const mg_ctx_s &c)
{
    int64_t vs = 0;
    for (const ProbBuf &pb : c.probs) vs = std::max<int64_t>(vs, pb.lev[0].plane);
    return (vs + 63) / 64 * 64;
}

size_t workspace_doubles(int64_t vs, int m, size_t *vec_part)
{
    *vec_part = (size_t)(2 * m + 4) * vs;
    return *vec_part + (size_t)(m + 2) * kKrylovBlocks + 4 * (size_t)(m + 2);
}

mg_status ensure_workspace(mg_ctx_s &c, int m, Workspace &ws)
{
    const int64_t vs = vector_stride(c);
    if (!(c.kr_restart >= m && c.kr_vec)) {
        size_t vec_part = 0;
        const size_t total = workspace_doubles(vs, m, &vec_part);
        void *p = nullptr;
        MG_TRY(c.arena.alloc(&p, vec_part * sizeof(double)));
        c.kr_vec = (double *)p;
        MG_TRY(c.arena.alloc(&p, (total - vec_part) * sizeof(double)));
        c.kr_small = (double *)p;
        c.kr_restart = m;
    }
    ws.vec = c.kr_vec;
    ws.small = c.kr_small;
    ws.restart = c.kr_restart;
    ws.vs = vs;
    return MG_OK;
}

struct Result {
    int iters = 0, status = MG_NOT_CONVERGED;
    double relres = 1.0;
};

mg_status fgmres_problem(mg_ctx_s &c, int p, double rtol, int maxit, int m, const Workspace &ws, double *hist,
                         Result &res, hipStream_t st)
{
    const ProbBuf &pb = c.probs[p];
    const LevelBuf &L0 = pb.lev[0];
    const int n = pb.n, P = L0.P;
    const int64_t plane = L0.plane, bytes = plane * (int64_t)sizeof(double);
    const int64_t vs = ws.vs;
    const int mw = ws.restart;
    double *V = ws.vec, *Z = V + (int64_t)(mw + 1) * vs, *w = Z + (int64_t)mw * vs, *X = w + vs, *r = X + vs;
    double *partial = ws.small, *h1 = partial + (int64_t)(mw + 2) * kKrylovBlocks, *h2 = h1 + (mw + 2),
           *ydev = h2 + (mw + 2), *nrm = ydev + (mw + 2);
    const bool mixed = c.opt.precision != MG_PREC_FP64;

    std::vector<char> act(c.nprob, 0);
    act[p] = 1;
    MG_TRY(ctx_set_live(c, act));
    launch_activate(c.d_state, c.nprob, st);
    launch_zero_f64(X, plane, st);

    auto norm_to_host = [&](const double *x, double &out) -> mg_status {
        launch_kr_dots(n, P, x, x, 0, 1, partial, nrm, 1, st);
        MG_HIP(hipMemcpyAsync(&out, nrm, sizeof(double), hipMemcpyDeviceToHost, st));
        MG_HIP(hipStreamSynchronize(st));
        return MG_OK;
    };
    double fnorm = 0.0;
    MG_TRY(norm_to_host(pb.f, fnorm));
    MG_HIP(hipMemcpyAsync(r, pb.f, bytes, hipMemcpyDeviceToDevice, st));
    double beta = fnorm;
    if (hist) hist[0] = fnorm > 0.0 ? 1.0 : 0.0;
    res = Result();
    if (!(fnorm > 0.0) || beta <= rtol * fnorm) {
        res.status = MG_OK;
        res.relres = 0.0;
        return MG_OK;
    }
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m), c1(m + 1), c2(m + 1);
    while (res.iters < maxit) {
        // v_0 = r / beta (nrm holds ||r|| from the last norm)
        launch_kr_scale(n, P, r, nrm, V, st);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int k = 0;  // columns in this cycle
        for (int j = 0; j < m; ++j) {
            double *vj = V + (int64_t)j * vs, *zj = Z + (int64_t)j * vs;
            // z_j = M v_j: the cycle reads level-0 r and adds its correction to u
            if (mixed)
                launch_to_f32(plane, vj, (float *)L0.r, st);
            else
                MG_HIP(hipMemcpyAsync(L0.r, vj, bytes, hipMemcpyDeviceToDevice, st));
            launch_zero_f64(pb.u, plane, st);
            ctx_enqueue_cycle(c, st);
            MG_HIP(hipMemcpyAsync(zj, pb.u, bytes, hipMemcpyDeviceToDevice, st));
            // w = A z_j, orthogonalised against v_0..v_j twice
            launch_kr_apply(n, P, plane, L0.A64, zj, nullptr, 1.0, w, st);
            launch_kr_dots(n, P, w, V, vs, j + 1, partial, h1, 0, st);
            launch_kr_update(n, P, w, V, vs, j + 1, h1, st);
            launch_kr_dots(n, P, w, V, vs, j + 1, partial, h2, 0, st);
            launch_kr_update(n, P, w, V, vs, j + 1, h2, st);
            launch_kr_dots(n, P, w, w, 0, 1, partial, nrm, 1, st);
            launch_kr_scale(n, P, w, nrm, V + (int64_t)(j + 1) * vs, st);  // v_{j+1} (unused if the cycle ends)
            MG_HIP(hipMemcpyAsync(c1.data(), h1, sizeof(double) * (j + 1), hipMemcpyDeviceToHost, st));
            MG_HIP(hipMemcpyAsync(c2.data(), h2, sizeof(double) * (j + 1), hipMemcpyDeviceToHost, st));
            double hn = 0.0;
            MG_HIP(hipMemcpyAsync(&hn, nrm, sizeof(double), hipMemcpyDeviceToHost, st));
            MG_HIP(hipStreamSynchronize(st));
            // column j of the Hessenberg, rotated by the previous Givens rotations
            double *col = &H[(size_t)j * (m + 1)];
            for (int i = 0; i <= j; ++i) col[i] = c1[i] + c2[i];
            col[j + 1] = hn;
            for (int i = 0; i < j; ++i) {
                const double a = cs[i] * col[i] + sn[i] * col[i + 1];
                col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
                col[i] = a;
            }
            const double d = std::hypot(col[j], col[j + 1]);
            cs[j] = d > 0.0 ? col[j] / d : 1.0;
            sn[j] = d > 0.0 ? col[j + 1] / d : 0.0;
            col[j] = d;
            col[j + 1] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            k = j + 1;
            res.iters += 1;
            const double est = std::fabs(g[j + 1]);
            if (hist) hist[res.iters] = est / fnorm;
            if (est <= rtol * fnorm || res.iters >= maxit || !(hn > 0.0)) break;
        }
        // y = R^{-1} g, u += Z y
        for (int i = k - 1; i >= 0; --i) {
            double s = g[i];
            for (int q = i + 1; q < k; ++q) s -= H[(size_t)q * (m + 1) + i] * y[q];
            const double dii = H[(size_t)i * (m + 1) + i];
            y[i] = dii != 0.0 ? s / dii : 0.0;
        }
        MG_HIP(hipMemcpyAsync(ydev, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, st));
        launch_kr_combine(n, P, X, Z, vs, k, ydev, st);
        // true residual of the new iterate
        launch_kr_apply(n, P, plane, L0.A64, X, pb.f, -1.0, r, st);
        MG_TRY(norm_to_host(r, beta));
        res.relres = beta / fnorm;
        if (!std::isfinite(beta)) {
            res.status = MG_ERR_DIVERGED;
            break;
        }
        if (beta <= rtol * fnorm) {
            res.status = MG_OK;
            break;
        }
    }
    // the iterate into pb.u, where copy-out finds it
    MG_HIP(hipMemcpyAsync(pb.u, X, bytes, hipMemcpyDeviceToDevice, st));
    return MG_OK;
}

// The solve of every problem with the given workspace (the body of both entry points).
mg_status fgmres_all(mg_ctx_s &c, const double *const *f, double *const *u, double rtol, int32_t maxit,
                     int32_t restart, const Workspace &ws, int32_t *iters, double *relres, int32_t *status,
                     double *history)
{
    MG_TRY(c.join.enter());
    hipStream_t st = c.join.internal;
    MG_HIP(hipEventRecord(c.t0, st));
    std::vector<double> hist;
    if (history) hist.assign((size_t)c.nprob * (maxit + 1), 0.0);
    mg_status agg = MG_OK;
    for (int p = 0; p < c.nprob; ++p) {
        const ProbBuf &pb = c.probs[p];
        launch_copy_field(pb.n, 1, f[p], pb.n, (int64_t)pb.n * pb.n, pb.f, pb.lev[0].P, pb.lev[0].plane, st);
        Result r;
        MG_TRY(fgmres_problem(c, p, rtol, maxit, restart, ws, history ? &hist[(size_t)p * (maxit + 1)] : nullptr, r,
                              st));
        launch_copy_field(pb.n, 1, pb.u, pb.lev[0].P, pb.lev[0].plane, u[p], pb.n, (int64_t)pb.n * pb.n, st);
        if (iters) iters[p] = r.iters;
        if (relres) relres[p] = r.relres;
        if (status) status[p] = r.status;
        if (r.status == MG_ERR_DIVERGED) agg = MG_ERR_DIVERGED;
        else if (r.status == MG_NOT_CONVERGED && agg == MG_OK) agg = MG_NOT_CONVERGED;
    }
    MG_TRY(ctx_set_live(c, std::vector<char>(c.nprob, 1)));
    MG_HIP(hipEventRecord(c.t1, st));
    MG_HIP(hipGetLastError());
    MG_HIP(hipStreamSynchronize(st));
    float ms = 0.0f;
    MG_HIP(hipEventElapsedTime(&ms, c.t0, c.t1));
    c.last_ms = ms;
    if (history) std::copy(hist.begin(), hist.end(), history);
    MG_TRY(c.join.leave());
    return agg;
}

mg_status check_fgmres_args(mg_ctx ctx, const double *const *f, double *const *u, double rtol, int32_t maxit,
                            int32_t restart)
{
    MG_TRY(ctx_check(ctx));
    MG_TRY(ctx_check_vectors(ctx, f, u));
    if (!(rtol >= 0.0) || maxit < 0 || maxit > 100000000)
        return set_error(MG_ERR_ARG, "need rtol >= 0 and 0 <= maxit <= 1e8");
    if (restart < 1 || restart > 256) return set_error(MG_ERR_ARG, "restart must be in [1, 256]");
    return ctx_check_smoother(*ctx);
}

}  // namespace

extern "C" mg_status mg_solve_fgmres(mg_ctx ctx, const double *const *f, double *const *u, double rtol,
                                     int32_t maxit, int32_t restart, int32_t *iters, double *relres, int32_t *status,
                                     double *history)
{
    clear_error();
    MG_TRY(check_fgmres_args(ctx, f, u, rtol, maxit, restart));
    Workspace ws;
    MG_TRY(ensure_workspace(*ctx, restart, ws));
    return fgmres_all(*ctx, f, u, rtol, maxit, restart, ws, iters, relres, status, history);
}

extern "C" mg_status mg_solve_fgmres_noalloc(mg_ctx ctx, const double *const *f, double *const *u, double rtol,
                                             int32_t maxit, int32_t restart, int32_t *iters, double *relres,
                                             int32_t *status, double *history)
{
    clear_error();
    MG_TRY(check_fgmres_args(ctx, f, u, rtol, maxit, restart));
    Workspace ws;
    ws.vs = vector_stride(*ctx);
    ws.restart = restart;
    size_t vec_part = 0;
    const size_t need = workspace_doubles(ws.vs, restart, &vec_part) * sizeof(double);
    if (need > kKrylovStaticBytes)
        return set_error(MG_ERR_ARG,
                         "FGMRES(%d) on a finest grid of %lld values needs %zu bytes of workspace; the fixed "
                         "workspace holds %zu (use a smaller restart, or mg_solve_fgmres)",
                         restart, (long long)ws.vs, need, kKrylovStaticBytes);
    double *base = nullptr;
    const hipError_t e = krylov_static_workspace(&base);
    if (e != hipSuccess)
        return set_error(MG_ERR_DEVICE, "fixed FGMRES workspace: %s", hipGetErrorString(e));
    ws.vec = base;
    ws.small = base + vec_part;
    return fgmres_all(*ctx, f, u, rtol, maxit, restart, ws, iters, relres, status, history);
}
