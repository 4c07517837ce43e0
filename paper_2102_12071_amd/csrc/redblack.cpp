// Red-black coarsening (section 6.1) with damped Jacobi or the two-layer
// convolution smoother H = f2(f1) (section 6, "Neural networks"): the
// hierarchy, its V-cycle (Algorithm 1), the stationary solve and one step of
// the adaptive training (Algorithm 2) of a level's smoother.  FP64.
//
// A context holds one operator's hierarchy and batches of vectors: the solve
// runs several right-hand sides at once, the training step runs every
// instance together with its 18 forward-mode tangents (the derivatives of the
// state with respect to the weights), all as independent vectors of the same
// kernels.  Level footprints are worked out on the host from the transfer
// stencils (which offsets a Galerkin product can reach), the values on the
// device.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <set>
#include <utility>
#include <vector>

#include "internal.hpp"
#include "launch.hpp"
#include "redblack.hpp"

using namespace mg;

namespace {

constexpr int kInstVecs = kRBWeights + 1;  // state + one tangent per weight
constexpr int kMaxAlphaCycles = 64;

struct RBLevel {
    RBGeom g{};
    RBOffsets o{};
    double *A = nullptr;                                  // [K][N][P]
    double *r = nullptr, *e = nullptr, *s = nullptr, *t = nullptr;  // [cap][N][P]
    int cap = 0;
    double *w = nullptr;                                  // device [18] (stack weights)
    bool stack = false;
};

}  // namespace

struct mg_rb_s {
    int n = 0, nlev = 0;
    RBLevel lev[kRBMaxLevels];
    double *Ainv = nullptr;
    int m = 0;  // points of the last level
    int *d_flag = nullptr;
    // solve
    double *u = nullptr, *f = nullptr, *partial = nullptr, *rr = nullptr, *hist = nullptr;
    RBState *state = nullptr;
    int *act = nullptr;
    int solve_cap = 0;
    int64_t solve_vs = 0;
    size_t hist_cap = 0;
    // training (vectors of the trained level; grown on demand)
    int tr_level = -1, tr_cap = 0;
    double *TU = nullptr, *TF = nullptr, *TR = nullptr, *TA = nullptr, *TS = nullptr, *TC = nullptr,
           *TSTAR = nullptr, *tpart = nullptr, *tsum = nullptr, *tout = nullptr;
    int *tact = nullptr, *twant = nullptr;
    size_t tact_cap = 0;
    std::vector<int> host_act;
    Arena arena;
    StreamJoin join;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    double last_ms = 0.0;
};

namespace {

bool is_pow2m1(int n) { return n >= 1 && ((n + 1) & n) == 0; }

// The offsets a Galerkin product R A P can reach from the fine footprint (fine units in, coarse units
// out), as in the kernel: a over the restriction's five nodes, then the fine footprint, then the
// interpolation's reach back to a coarse node.
RBOffsets next_offsets(const RBOffsets &of, int fine_kind)
{
    const bool diag = fine_kind == kRBChecker;
    const int ax[5][2] = {{0, 0}, {1, 0}, {-1, 0}, {0, 1}, {0, -1}};
    const int dg[5][2] = {{0, 0}, {1, 1}, {-1, 1}, {1, -1}, {-1, -1}};
    const int(*T)[2] = diag ? dg : ax;
    std::set<std::pair<int, int>> out;  // (dy, dx), ordered
    for (int a = 0; a < 5; ++a)
        for (int c = 0; c < of.K; ++c) {
            const int bx = T[a][0] + of.dx[c], by = T[a][1] + of.dy[c];
            for (int q = 0; q < 5; ++q) {
                // b = q' (weight 1) or b = q' + T[q] (weight 1/4): q' = b - T[q]
                const int tx = bx - T[q][0], ty = by - T[q][1];
                if (diag) {
                    if ((tx & 1) || (ty & 1)) continue;  // both-odd to both-odd: even fine offsets
                    out.insert({ty / 2, tx / 2});
                } else {
                    if ((tx + ty) & 1) continue;  // black to black
                    out.insert({ty, tx});
                }
            }
        }
    RBOffsets o{};
    o.K = 0;
    o.kc = -1;
    for (const auto &d : out) {
        o.dy[o.K] = (int8_t)d.first;
        o.dx[o.K] = (int8_t)d.second;
        if (d.first == 0 && d.second == 0) o.kc = o.K;
        ++o.K;
    }
    return o;
}

mg_status check_rb(mg_rb h)
{
    if (!h) return set_error(MG_ERR_ARG, "red-black context is null");
    return MG_OK;
}

mg_status ensure_level_vectors(mg_rb_s &h, int from, int cap)
{
    for (int l = from; l < h.nlev; ++l) {
        RBLevel &L = h.lev[l];
        if (L.cap >= cap) continue;
        const size_t bytes = (size_t)cap * L.g.vs * sizeof(double);
        void *p = nullptr;
        MG_TRY(h.arena.alloc(&p, bytes));
        L.r = (double *)p;
        MG_TRY(h.arena.alloc(&p, bytes));
        L.e = (double *)p;
        MG_TRY(h.arena.alloc(&p, bytes));
        L.s = (double *)p;
        MG_TRY(h.arena.alloc(&p, bytes));
        L.t = (double *)p;
        L.cap = cap;
    }
    return MG_OK;
}

// e (+)= H src on level l for nvec vectors (src: the residual).
void smooth(mg_rb_s &h, int l, const double *src, bool accumulate, int nvec, const int *act, hipStream_t st)
{
    RBLevel &L = h.lev[l];
    if (L.stack) {
        launch_rb_conv(L.g, L.w, src, L.t, true, false, false, nvec, act, st);
        launch_rb_conv(L.g, L.w + 9, L.t, L.e, false, true, accumulate, nvec, act, st);
    } else {
        launch_rb_jacobi(L.g, L.A + (int64_t)L.o.kc * L.g.vs, 2.0 / 3.0, src, L.e, accumulate, nvec, act, st);
    }
}

// e_l = V(r_l) from level l (Algorithm 1, correction form).
void vcycle(mg_rb_s &h, int l, int nvec, const int *act, int nu1, int nu2, hipStream_t st)
{
    RBLevel &L = h.lev[l];
    if (l == h.nlev - 1) {
        launch_rb_coarse_apply(L.g, h.m, h.Ainv, L.r, L.e, nvec, act, st);
        return;
    }
    if (nu1 == 0) {
        launch_zero_f64(L.e, (int64_t)nvec * L.g.vs, st);
    } else {
        smooth(h, l, L.r, false, nvec, act, st);
        for (int q = 1; q < nu1; ++q) {
            launch_rb_residual(L.g, L.o, L.A, L.r, L.e, L.s, -1.0, nvec, act, st);
            smooth(h, l, L.s, true, nvec, act, st);
        }
    }
    RBLevel &C = h.lev[l + 1];
    launch_rb_residual(L.g, L.o, L.A, L.r, L.e, L.s, -1.0, nvec, act, st);
    launch_rb_restrict(L.g, C.g, L.s, C.r, nvec, act, st);
    vcycle(h, l + 1, nvec, act, nu1, nu2, st);
    launch_rb_prolong(L.g, C.g, C.e, L.e, nvec, act, st);
    for (int q = 0; q < nu2; ++q) {
        launch_rb_residual(L.g, L.o, L.A, L.r, L.e, L.s, -1.0, nvec, act, st);
        smooth(h, l, L.s, true, nvec, act, st);
    }
}

mg_status check_level(const mg_rb_s &h, int level, bool smoothing)
{
    if (level < 0 || level >= h.nlev || (smoothing && level == h.nlev - 1))
        return set_error(MG_ERR_ARG, "level %d out of range (levels 0..%d%s)", level, h.nlev - 1,
                         smoothing ? ", the last one has no smoother" : "");
    return MG_OK;
}

}  // namespace

extern "C" {

mg_status mg_rb_create(int32_t n, const double *stencil, int32_t nlevels, void *stream, mg_rb *out)
{
    clear_error();
    if (!out) return set_error(MG_ERR_ARG, "out is null");
    *out = nullptr;
    if (!stencil) return set_error(MG_ERR_ARG, "stencil is null");
    if (!is_pow2m1(n) || n < 1 || n > 8191) return set_error(MG_ERR_ARG, "n = %d must be 2^k - 1, <= 8191", n);
    if (nlevels < 1 || nlevels > kRBMaxLevels) return set_error(MG_ERR_ARG, "nlevels must be in [1, %d]", kRBMaxLevels);
    // shapes: full n, checkerboard n, full (n-1)/2, ...
    std::vector<std::pair<int, int>> shapes = {{n, kRBFull}};
    while ((int)shapes.size() < nlevels) {
        const auto [N, kind] = shapes.back();
        if (kind == kRBFull) {
            if (N < 3) return set_error(MG_ERR_ARG, "%d levels need a finer grid than n = %d", nlevels, n);
            shapes.push_back({N, kRBChecker});
        } else {
            shapes.push_back({(N - 1) / 2, kRBFull});
        }
    }
    const auto [Nl, kl] = shapes.back();
    const int m = kl == kRBFull ? Nl * Nl : (Nl * Nl + 1) / 2;
    if (m > kRBMaxCoarse)
        return set_error(MG_ERR_ARG, "the last level (%d x %d, %s) has %d points; at most %d are solved directly",
                         Nl, Nl, kl == kRBFull ? "full" : "checkerboard", m, kRBMaxCoarse);
    MG_TRY(require_device());
    mg_rb h = new mg_rb_s();
    auto fail = [&](mg_status s) {
        h->arena.release();
        h->join.destroy();
        delete h;
        return s;
    };
    mg_status s = h->join.init((hipStream_t)stream);
    if (s < 0) return fail(s);
    h->arena.stream = h->join.internal;
    h->n = n;
    h->nlev = nlevels;
    h->m = m;
    if (hipEventCreate(&h->t0) != hipSuccess || hipEventCreate(&h->t1) != hipSuccess)
        return fail(set_error(MG_ERR_DEVICE, "hipEventCreate failed"));
    for (int l = 0; l < nlevels; ++l) {
        RBLevel &L = h->lev[l];
        L.g.N = shapes[l].first;
        L.g.kind = shapes[l].second;
        L.g.P = L.g.N + 1;
        L.g.vs = (int64_t)L.g.N * L.g.P;
        if (l == 0) {
            L.o.K = 9;
            L.o.kc = 4;
            for (int c = 0; c < 9; ++c) {
                L.o.dx[c] = (int8_t)(c % 3 - 1);
                L.o.dy[c] = (int8_t)(c / 3 - 1);
            }
        } else {
            L.o = next_offsets(h->lev[l - 1].o, h->lev[l - 1].g.kind);
            if (L.o.K > kRBMaxOffsets || L.o.kc < 0) return fail(set_error(MG_ERR_ARG, "footprint overflow"));
        }
        void *p = nullptr;
        if ((s = h->arena.alloc(&p, (size_t)L.o.K * L.g.vs * sizeof(double))) < 0) return fail(s);
        L.A = (double *)p;
        if ((s = h->arena.alloc(&p, kRBWeights * sizeof(double))) < 0) return fail(s);
        L.w = (double *)p;
    }
    void *p = nullptr;
    if ((s = h->arena.alloc(&p, (size_t)kRBMaxCoarse * kRBMaxCoarse * sizeof(double))) < 0) return fail(s);
    h->Ainv = (double *)p;
    if ((s = h->arena.alloc(&p, sizeof(int))) < 0) return fail(s);
    h->d_flag = (int *)p;
    hipStream_t st = h->join.internal;
    if ((s = h->join.enter()) < 0) return fail(s);
    const RBLevel &L0 = h->lev[0];
    launch_copy_field(n, 9, stencil, n, (int64_t)n * n, L0.A, L0.g.P, L0.g.vs, st);
    launch_rb_validate(L0.g, L0.A, h->d_flag, st);
    for (int l = 0; l + 1 < nlevels; ++l)
        launch_rb_galerkin(h->lev[l].g, h->lev[l].o, h->lev[l].A, h->lev[l + 1].g, h->lev[l + 1].o,
                           h->lev[l + 1].A, st);
    const RBLevel &Ll = h->lev[nlevels - 1];
    launch_rb_coarse_factor(Ll.g, Ll.o, Ll.A, m, h->Ainv, h->d_flag, st);
    int flag = 0;
    if (hipGetLastError() != hipSuccess || hipMemcpyAsync(&flag, h->d_flag, sizeof flag, hipMemcpyDeviceToHost, st) !=
                                               hipSuccess || hipStreamSynchronize(st) != hipSuccess)
        return fail(set_error(MG_ERR_DEVICE, "red-black set-up failed"));
    if (flag & 3)
        return fail(set_error(MG_ERR_ARG, "stencil %s", (flag & 2) ? "has a non-positive centre entry"
                                                                      : "couples to nodes off the grid (or is not finite)"));
    if (flag & 8) return fail(set_error(MG_ERR_ARG, "the last level's operator is not positive definite"));
    if ((s = h->join.leave()) < 0) return fail(s);
    *out = h;
    return MG_OK;
}

mg_status mg_rb_destroy(mg_rb h)
{
    clear_error();
    if (!h) return MG_OK;
    h->join.destroy();
    h->arena.release();
    if (h->t0) (void)hipEventDestroy(h->t0);
    if (h->t1) (void)hipEventDestroy(h->t1);
    delete h;
    return MG_OK;
}

mg_status mg_rb_level(mg_rb h, int32_t level, int32_t *N, int32_t *checker, int32_t *noffsets)
{
    clear_error();
    MG_TRY(check_rb(h));
    MG_TRY(check_level(*h, level, false));
    const RBLevel &L = h->lev[level];
    if (N) *N = L.g.N;
    if (checker) *checker = L.g.kind;
    if (noffsets) *noffsets = L.o.K;
    return MG_OK;
}

mg_status mg_rb_get_stencil(mg_rb h, int32_t level, int32_t *offsets, double *out)
{
    clear_error();
    MG_TRY(check_rb(h));
    MG_TRY(check_level(*h, level, false));
    const RBLevel &L = h->lev[level];
    if (offsets)
        for (int c = 0; c < L.o.K; ++c) {
            offsets[2 * c] = L.o.dx[c];
            offsets[2 * c + 1] = L.o.dy[c];
        }
    if (out) {
        MG_TRY(h->join.enter());
        launch_copy_field(L.g.N, L.o.K, L.A, L.g.P, L.g.vs, out, L.g.N, (int64_t)L.g.N * L.g.N, h->join.internal);
        MG_HIP(hipGetLastError());
        MG_TRY(h->join.leave());
    }
    return MG_OK;
}

mg_status mg_rb_set_smoother(mg_rb h, int32_t level, const double *phi, double a_ref)
{
    clear_error();
    MG_TRY(check_rb(h));
    MG_TRY(check_level(*h, level, true));
    RBLevel &L = h->lev[level];
    if (!phi) {
        L.stack = false;
        return MG_OK;
    }
    if (!(a_ref >= 0.0) || !std::isfinite(a_ref)) return set_error(MG_ERR_ARG, "a_ref must be finite and >= 0");
    double w[kRBWeights];
    for (int q = 0; q < kRBWeights; ++q) {
        if (!std::isfinite(phi[q])) return set_error(MG_ERR_ARG, "weight %d is not finite", q);
        w[q] = phi[q];
    }
    MG_TRY(h->join.enter());
    hipStream_t st = h->join.internal;
    if (a_ref > 0.0) {  // f1 times a_ref / a_C of this level's middle node
        const int mid = L.g.N / 2;
        double ac = 0.0;
        MG_HIP(hipMemcpyAsync(&ac, L.A + (int64_t)L.o.kc * L.g.vs + (int64_t)mid * L.g.P + mid, sizeof(double),
                              hipMemcpyDeviceToHost, st));
        MG_HIP(hipStreamSynchronize(st));
        if (!(ac > 0.0)) return set_error(MG_ERR_ARG, "level %d has no positive centre entry at its middle node", level);
        for (int q = 0; q < 9; ++q) w[q] *= a_ref / ac;
    }
    MG_HIP(hipMemcpyAsync(L.w, w, kRBWeights * sizeof(double), hipMemcpyHostToDevice, st));
    MG_HIP(hipStreamSynchronize(st));
    L.stack = true;
    return h->join.leave();
}

mg_status mg_rb_vcycle(mg_rb h, int32_t level, int32_t nvec, const double *r, double *e, int32_t nu_pre,
                       int32_t nu_post)
{
    clear_error();
    MG_TRY(check_rb(h));
    MG_TRY(check_level(*h, level, false));
    if (nvec < 1 || nvec > 65535) return set_error(MG_ERR_ARG, "nvec must be in [1, 65535]");
    if (!r || !e) return set_error(MG_ERR_ARG, "null vector");
    if (nu_pre < 0 || nu_pre > 8 || nu_post < 0 || nu_post > 8) return set_error(MG_ERR_ARG, "sweeps in [0, 8]");
    mg_rb_s &c = *h;
    MG_TRY(ensure_level_vectors(c, level, nvec));
    MG_TRY(c.join.enter());
    hipStream_t st = c.join.internal;
    RBLevel &L = c.lev[level];
    launch_rb_copy_in(L.g, r, L.r, L.g.vs, nvec, st);
    vcycle(c, level, nvec, nullptr, nu_pre, nu_post, st);
    launch_rb_copy_out(L.g, L.e, e, nvec, st);
    MG_HIP(hipGetLastError());
    return c.join.leave();
}

mg_status mg_rb_solve(mg_rb h, int32_t level, int32_t nvec, const double *f, double *u, double rtol, int32_t maxit,
                      int32_t nu_pre, int32_t nu_post, int32_t *iters, double *relres, int32_t *status,
                      double *history)
{
    clear_error();
    MG_TRY(check_rb(h));
    MG_TRY(check_level(*h, level, false));
    if (nvec < 1 || nvec > 65535) return set_error(MG_ERR_ARG, "nvec must be in [1, 65535]");
    if (!f || !u) return set_error(MG_ERR_ARG, "null vector");
    if (!(rtol >= 0.0) || maxit < 0 || maxit > 100000000) return set_error(MG_ERR_ARG, "need rtol >= 0, maxit >= 0");
    if (nu_pre < 0 || nu_pre > 8 || nu_post < 0 || nu_post > 8) return set_error(MG_ERR_ARG, "sweeps in [0, 8]");
    mg_rb_s &c = *h;
    RBLevel &L = c.lev[level];
    MG_TRY(ensure_level_vectors(c, level, nvec));
    const int nb = rb_norm_blocks(L.g.N);
    if (c.solve_cap < nvec || c.solve_vs < L.g.vs) {
        void *p = nullptr;
        MG_TRY(c.arena.alloc(&p, (size_t)nvec * L.g.vs * sizeof(double)));
        c.u = (double *)p;
        MG_TRY(c.arena.alloc(&p, (size_t)nvec * L.g.vs * sizeof(double)));
        c.f = (double *)p;
        MG_TRY(c.arena.alloc(&p, (size_t)nvec * nb * sizeof(double)));
        c.partial = (double *)p;
        MG_TRY(c.arena.alloc(&p, (size_t)nvec * sizeof(double)));
        c.rr = (double *)p;
        MG_TRY(c.arena.alloc(&p, (size_t)nvec * sizeof(RBState)));
        c.state = (RBState *)p;
        MG_TRY(c.arena.alloc(&p, (size_t)nvec * sizeof(int)));
        c.act = (int *)p;
        c.solve_cap = nvec;
        c.solve_vs = L.g.vs;
    }
    const int stride = maxit + 1;
    if (history && (size_t)nvec * stride > c.hist_cap) {
        void *p = nullptr;
        MG_TRY(c.arena.alloc(&p, (size_t)nvec * stride * sizeof(double)));
        c.hist = (double *)p;
        c.hist_cap = (size_t)nvec * stride;
    }
    MG_TRY(c.join.enter());
    hipStream_t st = c.join.internal;
    MG_HIP(hipEventRecord(c.t0, st));
    launch_rb_copy_in(L.g, f, c.f, L.g.vs, nvec, st);
    launch_zero_f64(c.u, (int64_t)nvec * L.g.vs, st);
    if (history) launch_zero_f64(c.hist, (int64_t)nvec * stride, st);
    // ||f||: the residual of u = 0
    launch_rb_outer(L.g, L.o, L.A, c.f, c.u, L.r, c.partial, nvec, nullptr, st);
    launch_rb_sum(c.partial, nb, c.rr, nvec, st);
    launch_rb_check(c.rr, c.state, c.act, rtol, maxit, history ? c.hist : nullptr, stride, 1, nvec, st);
    std::vector<RBState> hs(nvec);
    constexpr int kEvery = 16;
    for (int64_t done = 0;; done += kEvery) {
        for (int q = 0; q < kEvery; ++q) {
            launch_rb_outer(L.g, L.o, L.A, c.f, c.u, L.r, c.partial, nvec, c.act, st);
            launch_rb_sum(c.partial, nb, c.rr, nvec, st);
            launch_rb_check(c.rr, c.state, c.act, rtol, maxit, history ? c.hist : nullptr, stride, 0, nvec, st);
            vcycle(c, level, nvec, c.act, nu_pre, nu_post, st);
            launch_rb_axpy(L.g, L.e, c.u, nvec, c.act, st);
        }
        MG_HIP(hipMemcpyAsync(hs.data(), c.state, sizeof(RBState) * nvec, hipMemcpyDeviceToHost, st));
        MG_HIP(hipStreamSynchronize(st));
        bool any = false;
        for (const RBState &s : hs) any |= s.active != 0;
        if (!any || done > (int64_t)maxit + 2) break;
    }
    launch_rb_copy_out(L.g, c.u, u, nvec, st);
    MG_HIP(hipEventRecord(c.t1, st));
    MG_HIP(hipGetLastError());
    MG_HIP(hipStreamSynchronize(st));
    float ms = 0.0f;
    MG_HIP(hipEventElapsedTime(&ms, c.t0, c.t1));
    c.last_ms = ms;
    if (history) MG_HIP(hipMemcpy(history, c.hist, sizeof(double) * nvec * stride, hipMemcpyDeviceToHost));
    mg_status agg = MG_OK;
    for (int v = 0; v < nvec; ++v) {
        const int stt = hs[v].active ? MG_NOT_CONVERGED : hs[v].status;
        if (iters) iters[v] = hs[v].iters;
        if (relres) relres[v] = hs[v].relres;
        if (status) status[v] = stt;
        if (stt == MG_ERR_DIVERGED) agg = MG_ERR_DIVERGED;
        else if (stt == MG_NOT_CONVERGED && agg == MG_OK) agg = MG_NOT_CONVERGED;
    }
    MG_TRY(c.join.leave());
    return agg;
}

mg_status mg_rb_last_solve_ms(mg_rb h, double *ms)
{
    clear_error();
    MG_TRY(check_rb(h));
    if (!ms) return set_error(MG_ERR_ARG, "ms is null");
    *ms = h->last_ms;
    return MG_OK;
}

mg_status mg_rb_alpha_step(mg_rb h, int32_t level, double *phi, double *adam_m, double *adam_v, int32_t t,
                           int32_t B, const int32_t *k, const double *f, const double *u0, const double *u_star,
                           const mg_train_opts *o_in, double *loss, double *losses, double *grad)
{
    clear_error();
    MG_TRY(check_rb(h));
    MG_TRY(check_level(*h, level, true));
    if (!phi || !k || !f || !u0 || !u_star || !loss) return set_error(MG_ERR_ARG, "null argument");
    if (B < 1 || (int64_t)B * kInstVecs > 65535) return set_error(MG_ERR_ARG, "B must be in [1, %d]", 65535 / kInstVecs);
    mg_train_opts o;
    if (o_in)
        o = *o_in;
    else
        mg_train_opts_default(&o);
    if (o.apply_update && (!adam_m || !adam_v || t < 1))
        return set_error(MG_ERR_ARG, "an update needs the Adam moments and a step number t >= 1");
    int kmax = 0;
    for (int b = 0; b < B; ++b) {
        if (k[b] < 1 || k[b] > kMaxAlphaCycles)
            return set_error(MG_ERR_ARG, "k[%d] = %d must be in [1, %d]", b, k[b], kMaxAlphaCycles);
        kmax = std::max(kmax, k[b]);
    }
    mg_rb_s &c = *h;
    const RBLevel &L = c.lev[level];
    const RBGeom &g = L.g;
    const int V = B * kInstVecs;
    const int64_t vs = g.vs, is = (int64_t)kInstVecs * vs;  // instance stride
    const int nb = rb_norm_blocks(g.N);
    MG_TRY(ensure_level_vectors(c, level + 1, V));
    if (c.tr_level != level || c.tr_cap < V) {
        const size_t bytes = (size_t)V * vs * sizeof(double);
        void *p = nullptr;
        double **bufs[] = {&c.TU, &c.TF, &c.TR, &c.TA, &c.TS, &c.TC};
        for (double **q : bufs) {
            MG_TRY(c.arena.alloc(&p, bytes));
            *q = (double *)p;
        }
        MG_TRY(c.arena.alloc(&p, (size_t)B * vs * sizeof(double)));
        c.TSTAR = (double *)p;
        MG_TRY(c.arena.alloc(&p, (size_t)V * nb * sizeof(double)));
        c.tpart = (double *)p;
        MG_TRY(c.arena.alloc(&p, (size_t)V * sizeof(double)));
        c.tsum = (double *)p;
        MG_TRY(c.arena.alloc(&p, (size_t)(1 + B + kRBWeights) * sizeof(double)));
        c.tout = (double *)p;
        c.tr_level = level;
        c.tr_cap = V;
    }
    const size_t nact = (size_t)kmax * V + (size_t)kmax * B;
    if (nact > c.tact_cap) {
        void *p = nullptr;
        MG_TRY(c.arena.alloc(&p, nact * sizeof(int)));
        c.tact = (int *)p;
        c.tact_cap = nact;
    }
    // cycle q (0-based) runs the instances with k > q; after it, those with k == q + 1 are scored
    c.host_act.assign(nact, 0);
    for (int q = 0; q < kmax; ++q)
        for (int b = 0; b < B; ++b) {
            for (int v = 0; v < kInstVecs; ++v) c.host_act[(size_t)q * V + b * kInstVecs + v] = k[b] > q;
            c.host_act[(size_t)kmax * V + (size_t)q * B + b] = k[b] == q + 1;
        }
    c.twant = c.tact + (size_t)kmax * V;
    MG_TRY(c.join.enter());
    hipStream_t st = c.join.internal;
    MG_HIP(hipMemcpyAsync(c.tact, c.host_act.data(), nact * sizeof(int), hipMemcpyHostToDevice, st));
    // state rows: u0 and f; tangent rows: zero (u0 and f do not depend on the weights)
    launch_zero_f64(c.TU, (int64_t)V * vs, st);
    launch_zero_f64(c.TF, (int64_t)V * vs, st);
    launch_rb_copy_in(g, u0, c.TU, is, B, st);
    launch_rb_copy_in(g, f, c.TF, is, B, st);
    launch_rb_copy_in(g, u_star, c.TSTAR, vs, B, st);
    const RBLevel &C = c.lev[level + 1];
    // H x for every row (conv1 into TC, conv2 into y), then the weights' tangent sources for the
    // state rows: y's tangent j += d(H x_state)/d w_j
    auto H_tangent = [&](const double *x, double *y, const int *act) {
        launch_rb_conv(g, phi, x, c.TC, true, false, false, V, act, st);
        launch_rb_conv(g, phi + 9, c.TC, y, false, true, false, V, act, st);
        launch_rb_dH(g, phi, x, is, c.TC, is, y + vs, is, vs, B, act, kInstVecs, st);
    };
    for (int q = 0; q < kmax; ++q) {
        const int *act = c.tact + (size_t)q * V;
        // r = f - A u
        launch_rb_residual(g, L.o, L.A, c.TF, c.TU, c.TR, -1.0, V, act, st);
        // a = H r
        H_tangent(c.TR, c.TA, act);
        // s = r - A a
        launch_rb_residual(g, L.o, L.A, c.TR, c.TA, c.TS, -1.0, V, act, st);
        // t = a + P Psi_c(R s): one V(1,1) cycle of the coarser levels for every row
        launch_rb_restrict(g, C.g, c.TS, C.r, V, act, st);
        vcycle(c, level + 1, V, act, 1, 1, st);
        launch_rb_prolong(g, C.g, C.e, c.TA, V, act, st);
        // q = r - A t;  u += t + H q
        launch_rb_residual(g, L.o, L.A, c.TR, c.TA, c.TS, -1.0, V, act, st);
        launch_rb_axpy(g, c.TA, c.TU, V, act, st);
        H_tangent(c.TS, c.TR, act);
        launch_rb_axpy(g, c.TR, c.TU, V, act, st);
        // instances whose k cycles are done: ||u - u*||^2 and <du/dw_j, u - u*>
        launch_rb_alpha_dots(g, c.TU, is, c.TSTAR, c.tpart, B, c.twant + (size_t)q * B, st);
    }
    launch_rb_sum(c.tpart, nb, c.tsum, V, st);
    launch_rb_alpha_final(c.tsum, B, c.tout, st);
    std::vector<double> hout(1 + B + kRBWeights);
    MG_HIP(hipMemcpyAsync(hout.data(), c.tout, hout.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    MG_HIP(hipStreamSynchronize(st));
    bool finite = true;
    for (double x : hout) finite &= std::isfinite(x);
    if (finite && o.apply_update)
        launch_rb_adam(kRBWeights, phi, adam_m, adam_v, c.tout + 1 + B, t, o.lr, o.beta1, o.beta2, o.adam_eps, st);
    MG_HIP(hipGetLastError());
    MG_HIP(hipStreamSynchronize(st));
    *loss = hout[0];
    if (losses) std::copy(hout.begin() + 1, hout.begin() + 1 + B, losses);
    if (grad) std::copy(hout.begin() + 1 + B, hout.end(), grad);
    MG_TRY(c.join.leave());
    if (!finite) return set_error(MG_ERR_DIVERGED, "loss or gradient is not finite (weights unchanged)");
    return MG_OK;
}

}  // extern "C"
