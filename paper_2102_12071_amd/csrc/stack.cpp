// Entry points of the convolution-stack smoother (the constant-coefficient
// alpha-CNN of section 5, full coarsening): installing a level's weights,
// applying the stack, and its adaptive training step (Algorithm 2).
//
// Training step, per cycle (all instances of the stage at once, FP64):
//     r = f - A u,  a = H r,  s = r - A a,  t = a + P Psi_c(R s),
//     q = r - A t,  u = u + t + H q,
// loss L = (1/B) sum_b ||u_k - u*||_2.  The adjoint pass is the one of the
// per-point form (A symmetric, the adjoint of Psi_c the coarse cycle with every
// smoother transposed) with H^T the stack of turned kernels in reverse order.
// Each application y = H x adds to the weight gradient, for the adjoint state
// g of y: layer L's kernel gets the correlation of x_L = f_L(..f_1(x)) with
// g_L = f_{L+2}^T(..f_5^T(g)) (f6: of x with g); the intermediates are
// recomputed from x.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "alpha.hpp"
#include "internal.hpp"
#include "stack.hpp"

using namespace mg;

namespace {

constexpr int kMaxCycles = 64;

// state vectors, adjoint vectors, and the gradient's intermediates x1..x4, g0..g3
enum { kU, kF, kUs, kA, kS, kT, kLam, kDq, kDt, kDs, kDa, kDr, kX1, kX2, kX3, kX4, kG0, kG1, kG2, kG3, kNumVec };

struct Work {
    AlphaProb *probs;  // device [B]
    int *active;       // device [kmax][B]
    double *dist;      // device [B]
    double *wT;        // device [54]
    double *grad;      // device [54]
    double *part;      // device [B][blocks][54]
    double *vec;       // [kNumVec + 2 kmax][B * vs]
    size_t bytes;
};

Work carve(char *base, int B, int kmax, int n, int64_t vs)
{
    Carve c{base};
    Work w;
    w.probs = c.take<AlphaProb>(B);
    w.active = c.take<int>((size_t)kmax * B);
    w.dist = c.take<double>(B);
    w.wT = c.take<double>(kStackWeights);
    w.grad = c.take<double>(kStackWeights);
    w.part = c.take<double>((size_t)B * stack_wgrad_blocks(n) * kStackWeights);
    w.vec = c.take<double>((size_t)(kNumVec + 2 * kmax) * B * vs);
    w.bytes = c.off;
    return w;
}

// Writes a level's weights: half 0 (before the coarse correction), 1 (after), or both (-1).
mg_status set_stack_half(mg_ctx ctx, int32_t prob, int32_t level, const double *phi, int32_t transpose,
                         int32_t normalised, int half)
{
    clear_error();
    MG_TRY(ctx_check(ctx));
    if (ctx->opt.smoother != MG_SMOOTHER_STACK) return set_error(MG_ERR_STATE, "the context's smoother is not the stack");
    if (prob < 0 || prob >= ctx->nprob) return set_error(MG_ERR_ARG, "problem %d out of range", prob);
    ProbBuf &pb = ctx->probs[prob];
    if (level < 0 || level + 1 >= pb.nlev)
        return set_error(MG_ERR_ARG, "level %d has no smoother (levels 0..%d)", level, pb.nlev - 2);
    if (!phi) return set_error(MG_ERR_ARG, "phi is null");
    if (transpose != 0 && transpose != 1) return set_error(MG_ERR_ARG, "transpose must be 0 or 1");
    if (normalised != 0 && normalised != 1) return set_error(MG_ERR_ARG, "normalised must be 0 or 1");
    LevelBuf &L = pb.lev[level];
    if (half == 1 && !L.phi_set) return set_error(MG_ERR_STATE, "set the level's stack (mg_set_stack) first");
    MG_TRY(ctx->join.enter());
    hipStream_t st = ctx->join.internal;
    double scale = 1.0;  // normalised weights: f5 and f6 over the level's mean centre entry
    if (normalised) {
        launch_stack_mean_centre(L.n, L.P, L.plane, L.A64, ctx->d_scalar, st);
        double ac = 0.0;
        MG_HIP(hipMemcpyAsync(&ac, ctx->d_scalar, sizeof ac, hipMemcpyDeviceToHost, st));
        MG_HIP(hipStreamSynchronize(st));
        if (!(ac > 0.0)) return set_error(MG_ERR_ARG, "level %d: the mean centre entry is not positive", level);
        scale = 1.0 / ac;
    }
    double w[2 * kStackWeights];
    for (int j = 0; j < kStackWeights; ++j) {
        const int Lr = j / 9, t = j % 9;
        w[j] = transpose ? phi[(Lr < 5 ? 4 - Lr : 5) * 9 + 8 - t] : phi[j];
        if (!std::isfinite(w[j])) return set_error(MG_ERR_ARG, "weight %d is not finite", j);
        if (j >= 4 * 9) w[j] *= scale;  // f5 and f6 (a turned stack keeps them as layers 5 and 6)
        w[kStackWeights + j] = w[j];
    }
    float wf[2 * kStackWeights];
    for (int j = 0; j < 2 * kStackWeights; ++j) wf[j] = (float)w[j];
    const bool fp64 = ctx->opt.precision == MG_PREC_FP64;
    const size_t es = fp64 ? sizeof(double) : sizeof(float);
    const int first = half == 1 ? kStackWeights : 0, count = half < 0 ? 2 * kStackWeights : kStackWeights;
    MG_HIP(hipMemcpyAsync((char *)L.phi + first * es, fp64 ? (const void *)w : (const void *)wf, count * es,
                          hipMemcpyHostToDevice, st));
    MG_HIP(hipStreamSynchronize(st));  // the host staging arrays end with this call
    L.phi_set = true;
    return ctx->join.leave();
}

}  // namespace

extern "C" {

mg_status mg_set_stack(mg_ctx ctx, int32_t prob, int32_t level, const double *phi, int32_t transpose,
                       int32_t normalised)
{
    return set_stack_half(ctx, prob, level, phi, transpose, normalised, -1);
}

mg_status mg_set_stack_post(mg_ctx ctx, int32_t prob, int32_t level, const double *phi, int32_t transpose,
                            int32_t normalised)
{
    return set_stack_half(ctx, prob, level, phi, transpose, normalised, 1);
}

mg_status mg_stack_apply(int32_t n, int32_t count, const double *phi, const double *x, double *y, int32_t accumulate,
                         void *stream)
{
    clear_error();
    if (n < 1 || n > 16383 || count < 0 || count > 65535) return set_error(MG_ERR_ARG, "n or count out of range");
    if (!phi || !x || !y) return set_error(MG_ERR_ARG, "null pointer");
    if (accumulate != 0 && accumulate != 1) return set_error(MG_ERR_ARG, "accumulate must be 0 or 1");
    const int64_t nn = (int64_t)n * n;
    const uintptr_t xa = (uintptr_t)x, ya = (uintptr_t)y, len = (uintptr_t)(nn * count) * sizeof(double);
    if (xa < ya + len && ya < xa + len) return set_error(MG_ERR_ARG, "x and y overlap");
    MG_TRY(require_device());
    if (count == 0) return MG_OK;
    launch_stack_vecs(x, y, nn, phi, n, n, count, accumulate != 0, nullptr, (hipStream_t)stream);
    MG_HIP(hipGetLastError());
    return MG_OK;
}

mg_status mg_stack_alpha_step(mg_ctx top, mg_ctx coarse, mg_ctx coarse_t, double *phi, double *adam_m,
                              double *adam_v, int32_t t, int32_t symmetric, const mg_alpha_batch *b,
                              const mg_train_opts *o_in, double *loss, double *losses, double *grad)
{
    clear_error();
    if (!top || !coarse || !coarse_t || !phi || !b) return set_error(MG_ERR_ARG, "null argument");
    if (symmetric != 0 && symmetric != 1) return set_error(MG_ERR_ARG, "symmetric must be 0 or 1");
    mg_train_opts o;
    if (o_in)
        o = *o_in;
    else
        mg_train_opts_default(&o);
    MG_TRY(check_train_opts(o));
    if (o.apply_update && (!adam_m || !adam_v || t < 1))
        return set_error(MG_ERR_ARG, "an update needs the Adam moments and a step number t >= 1");
    mg_ctx_s &c = *top;
    const int B = c.nprob;
    if (c.opt.precision != MG_PREC_FP64) return set_error(MG_ERR_ARG, "top must be an FP64 context");
    if (b->nprob != B) return set_error(MG_ERR_SHAPE, "batch has %d problems, top %d", b->nprob, B);
    if (!b->k || !b->f || !b->u0 || !b->u_star) return set_error(MG_ERR_ARG, "batch arrays must be non-null");
    if (b->dW) return set_error(MG_ERR_ARG, "the stack smoother has no smoother field: dW must be null");
    const int n = c.probs[0].n;
    int kmax = 0;
    for (int p = 0; p < B; ++p) {
        if (c.probs[p].n != n) return set_error(MG_ERR_SHAPE, "every problem of top must have the same n");
        if (b->k[p] < 1 || b->k[p] > kMaxCycles)
            return set_error(MG_ERR_ARG, "k[%d] = %d must be in [1, %d]", p, b->k[p], kMaxCycles);
        if (!b->f[p] || !b->u0[p] || !b->u_star[p]) return set_error(MG_ERR_ARG, "problem %d: null vector", p);
        kmax = std::max(kmax, b->k[p]);
    }
    if (c.probs[0].nlev < 2) return set_error(MG_ERR_SHAPE, "top needs a coarser level (n > coarsest_n)");
    MG_TRY(check_alpha_coarse(c, *coarse, "coarse"));
    MG_TRY(check_alpha_coarse(c, *coarse_t, "coarse_t"));
    if (coarse == top || coarse_t == top) return set_error(MG_ERR_ARG, "the coarse contexts must differ from top");

    const LevelBuf &L0 = c.probs[0].lev[0];
    const int P = L0.P;
    const int64_t plane = L0.plane, vs = (plane + 31) / 32 * 32;
    const Work need = carve(nullptr, B, kmax, n, vs);
    if (need.bytes > c.al_bytes) {
        MG_TRY(c.arena.alloc(&c.al_ws, need.bytes));
        c.al_bytes = need.bytes;
    }
    const Work w = carve((char *)c.al_ws, B, kmax, n, vs);

    // the coarse contexts' slot tables are rewritten synchronously: their streams must be idle
    MG_HIP(hipStreamSynchronize(coarse->join.internal));
    MG_HIP(hipStreamSynchronize(coarse_t->join.internal));
    MG_TRY(ctx_set_live(*coarse, std::vector<char>(B, 1)));
    MG_TRY(ctx_set_live(*coarse_t, std::vector<char>(B, 1)));
    MG_TRY(c.join.enter());
    hipStream_t st = c.join.internal;
    MG_HIP(hipStreamSynchronize(st));  // the previous step's table upload has been read

    std::vector<AlphaProb> probs(B);
    std::vector<int> active((size_t)kmax * B);
    for (int p = 0; p < B; ++p) {
        AlphaProb &a = probs[p];
        a.A = c.probs[p].lev[0].A64;
        a.H = nullptr;
        const mg_ctx_s *cc[2] = {coarse, coarse_t};
        for (int q = 0; q < 2; ++q) {
            a.rc[q] = (double *)cc[q]->probs[p].lev[0].r;
            a.uc[q] = cc[q]->probs[p].u;
        }
        for (int i = 0; i < kmax; ++i) active[(size_t)i * B + p] = i < b->k[p];
    }
    const size_t sz_probs = sizeof(AlphaProb) * B, sz_act = sizeof(int) * active.size();
    c.al_host.resize(sz_probs + sz_act);
    std::memcpy(c.al_host.data(), probs.data(), sz_probs);
    std::memcpy(c.al_host.data() + sz_probs, active.data(), sz_act);
    MG_HIP(hipMemcpyAsync(w.probs, c.al_host.data(), sz_probs, hipMemcpyHostToDevice, st));
    MG_HIP(hipMemcpyAsync(w.active, c.al_host.data() + sz_probs, sz_act, hipMemcpyHostToDevice, st));

    auto V = [&](int k) { return w.vec + (int64_t)k * B * vs; };
    auto Rv = [&](int i) { return V(kNumVec + i); };
    auto Qv = [&](int i) { return V(kNumVec + kmax + i); };
    const int64_t nn = (int64_t)n * n;
    for (int p = 0; p < B; ++p) {
        launch_copy_field(n, 1, b->u0[p], n, nn, V(kU) + p * vs, P, plane, st);
        launch_copy_field(n, 1, b->f[p], n, nn, V(kF) + p * vs, P, plane, st);
        launch_copy_field(n, 1, b->u_star[p], n, nn, V(kUs) + p * vs, P, plane, st);
    }
    launch_stack_transpose(phi, w.wT, st);
    const int nblk = stack_wgrad_blocks(n);
    launch_zero_f64(w.part, (int64_t)B * nblk * kStackWeights, st);
    auto coarse_cycle = [&](mg_ctx_s &cc) {
        launch_activate(cc.d_state, cc.nprob, st);
        ctx_enqueue_cycle(cc, st);
    };
    // y (+)= H x or H^T x
    auto H = [&](const double *x, double *y, bool transpose, bool acc, const int *act) {
        launch_stack_vecs(x, y, vs, transpose ? w.wT : phi, n, P, B, acc, act, st);
    };
    // the weight gradient of <g, H x>
    auto wgrad = [&](const double *g, const double *x, const int *act) {
        const double *xs[5] = {x, V(kX1), V(kX2), V(kX3), V(kX4)};
        for (int L = 0; L < 4; ++L) launch_stack_layer(xs[L], V(kX1 + L), vs, phi + 9 * L, false, n, P, B, act, st);
        const double *gs[5] = {V(kG0), V(kG1), V(kG2), V(kG3), g};
        for (int L = 3; L >= 0; --L)  // g_L = f_{L+2}^T g_{L+1}, with g_4 = g
            launch_stack_layer(gs[L + 1], V(kG0 + L), vs, phi + 9 * (L + 1), true, n, P, B, act, st);
        StackPairs pr;
        for (int L = 0; L < 5; ++L) {
            pr.g[L] = gs[L];
            pr.x[L] = xs[L];
        }
        pr.g[5] = g;
        pr.x[5] = x;
        launch_stack_wgrad(pr, vs, n, P, B, act, w.part, st);
    };

    // ---- forward
    for (int i = 0; i < kmax; ++i) {
        const int *act = w.active + (size_t)i * B;
        double *r = Rv(i), *q = Qv(i);
        launch_al_apply_A(w.probs, B, n, P, plane, vs, V(kU), V(kF), -1.0, r, act, st);        // r = f - A u
        H(r, V(kA), false, false, act);                                                         // a = H r
        launch_al_apply_A(w.probs, B, n, P, plane, vs, V(kA), r, -1.0, V(kS), act, st);        // s = r - A a
        launch_al_restrict(w.probs, 0, B, n, P, vs, V(kS), act, st);                             // r_c = R s
        coarse_cycle(*coarse);                                                                   // u_c = Psi_c(r_c)
        launch_al_prolong(w.probs, 0, B, n, P, vs, V(kA), V(kT), act, st);                     // t = a + P u_c
        launch_al_apply_A(w.probs, B, n, P, plane, vs, V(kT), r, -1.0, q, act, st);            // q = r - A t
        launch_al_axpy(B, n, P, vs, V(kU), 1.0, V(kT), V(kU), act, st);                         // u += t
        H(q, V(kU), symmetric != 0, true, act);                                                 // u += H' q
    }
    launch_al_dist(B, n, P, vs, V(kU), V(kUs), w.dist, st);
    std::vector<double> dist(B);
    MG_HIP(hipMemcpyAsync(dist.data(), w.dist, sizeof(double) * B, hipMemcpyDeviceToHost, st));
    MG_HIP(hipGetLastError());
    MG_HIP(hipStreamSynchronize(st));
    double total = 0.0;
    for (int p = 0; p < B; ++p) {
        if (!std::isfinite(dist[p])) {
            set_error(MG_ERR_DIVERGED, "instance %d: the loss is not finite (weights left unchanged)", p);
            (void)c.join.leave();
            return MG_ERR_DIVERGED;
        }
        total += dist[p];
    }

    // ---- adjoint: lam = dL/du_k, then back through the cycles
    launch_al_seed(B, n, P, plane, vs, V(kU), V(kUs), w.dist, 1.0 / B, V(kLam), nullptr, st);
    for (int i = kmax - 1; i >= 0; --i) {
        const int *act = w.active + (size_t)i * B;
        const double *r = Rv(i), *q = Qv(i);
        H(V(kLam), V(kDq), symmetric == 0, false, act);                                         // dq = H'^T lam
        if (symmetric)
            wgrad(q, V(kLam), act);  // post-smoothing H^T q: <lam, H^T q> = <q, H lam>
        else
            wgrad(V(kLam), q, act);  // post-smoothing H q
        launch_al_apply_A(w.probs, B, n, P, plane, vs, V(kDq), V(kLam), -1.0, V(kDt), act, st); // dt = lam - A dq
        launch_al_restrict(w.probs, 1, B, n, P, vs, V(kDt), act, st);                            // r_c = R dt
        coarse_cycle(*coarse_t);                                                                 // u_c = Psi_c^T(r_c)
        launch_al_prolong(w.probs, 1, B, n, P, vs, nullptr, V(kDs), act, st);                   // ds = P u_c
        launch_al_apply_A(w.probs, B, n, P, plane, vs, V(kDs), V(kDt), -1.0, V(kDa), act, st);  // da = dt - A ds
        wgrad(V(kDa), r, act);                                                                   // pre-smoothing H r
        launch_al_axpy(B, n, P, vs, V(kDs), 1.0, V(kDq), V(kDr), act, st);                      // dr = ds + dq
        H(V(kDa), V(kDr), true, true, act);                                                     // dr += H^T da
        launch_al_apply_A(w.probs, B, n, P, plane, vs, V(kDr), V(kLam), -1.0, V(kLam), act, st); // lam -= A dr
    }
    launch_stack_gsum(w.part, (int64_t)B * nblk, w.grad, st);
    if (o.apply_update) launch_stack_adam(phi, adam_m, adam_v, w.grad, t, o.lr, o.beta1, o.beta2, o.adam_eps, st);
    if (grad) MG_HIP(hipMemcpyAsync(grad, w.grad, sizeof(double) * kStackWeights, hipMemcpyDeviceToHost, st));
    MG_HIP(hipGetLastError());
    MG_HIP(hipStreamSynchronize(st));
    if (losses) std::copy(dist.begin(), dist.end(), losses);
    if (loss) *loss = total / B;
    return c.join.leave();
}

}  // extern "C"
