// Adaptive training step (Algorithm 2): the loss
//     L = (1/B) sum_b || Phi(u0_b, f_b, k_b) - u*_b ||_2
// of k_b cycles on the trained level, each a pre-smoothing with the network's
// smoother H, a coarse correction by one cycle Psi_c of the fixed coarser
// hierarchy and a post-smoothing with H, and its gradient with respect to
// the network's parameters, followed by an Adam update.
//
// Forward, per cycle (all problems of the stage at once):
//     r = f - A u,  a = H r,  s = r - A a,  t = a + P Psi_c(R s),
//     q = r - A t,  u = u + t + H q.
// Every step is linear in the state, so the gradient with respect to the
// smoother field is the reverse (adjoint) pass of the same steps: A is
// symmetric, H^T is a 5x5 gather with the taps read from the neighbours, and
// the adjoint of Psi_c is the same cycle with every smoother transposed (the
// context coarse_t).  dL/dH is accumulated from the outer products of the
// adjoint states with r and q, divided by a_C to give dL/dW, and the network
// backward (FP32, train.cpp) turns that into dL/dparams.  The loss and dL/dW
// are FP64.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "alpha.hpp"
#include "internal.hpp"
#include "launch.hpp"

using namespace mg;

namespace {

constexpr int kMaxCycles = 64;

// Vectors of the step, each B * vs doubles.
enum { kU, kF, kUs, kA, kS, kT, kLam, kDq, kDt, kDs, kDa, kDr, kNumVec };

struct Work {
    AlphaProb *probs;  // device [B]
    int *active;       // device [kmax][B]
    double **w64;      // device [B]
    double *dist;      // device [B]
    double *vec;       // [kNumVec + 2 kmax][B * vs]
    double *dH;        // [B][25][plane]
    float *dout;       // [B][25][n*n]
    double *dense_A;   // [B][9][n*n], the stencils in the training path's layout
    size_t bytes;
};

Work carve(char *base, int B, int kmax, int n, int64_t vs, int64_t plane)
{
    Carve c{base};
    Work w;
    w.probs = c.take<AlphaProb>(B);
    w.active = c.take<int>((size_t)kmax * B);
    w.w64 = c.take<double *>(B);
    w.dist = c.take<double>(B);
    w.vec = c.take<double>((size_t)(kNumVec + 2 * kmax) * B * vs);
    w.dH = c.take<double>((size_t)B * 25 * plane);
    w.dout = c.take<float>((size_t)B * 25 * n * n);
    w.dense_A = c.take<double>((size_t)B * 9 * n * n);
    w.bytes = c.off;
    return w;
}

}  // namespace

namespace mg {

mg_status check_alpha_coarse(const mg_ctx_s &top, const mg_ctx_s &c, const char *name)
{
    if (c.opt.precision != MG_PREC_FP64) return set_error(MG_ERR_ARG, "%s must be an FP64 context", name);
    if (c.nprob != top.nprob) return set_error(MG_ERR_SHAPE, "%s has %d problems, top %d", name, c.nprob, top.nprob);
    if (c.opt.nu_pre != c.opt.nu_post)
        return set_error(MG_ERR_ARG, "%s: the coarse cycle needs as many post- as pre-smoothing sweeps", name);
    bool smooths = false;  // a hierarchy of the coarsest level alone has no smoother to set
    for (const ProbBuf &q : c.probs) smooths = smooths || q.nlev > 1;
    if (smooths) MG_TRY(ctx_check_smoother(c));
    for (int p = 0; p < c.nprob; ++p) {
        const ProbBuf &t = top.probs[p], &q = c.probs[p];
        if (q.n != (t.n - 1) / 2 || q.nlev != t.nlev - 1)
            return set_error(MG_ERR_SHAPE, "%s problem %d: n = %d with %d levels, expected %d with %d", name, p, q.n,
                             q.nlev, (t.n - 1) / 2, t.nlev - 1);
    }
    return MG_OK;
}

}  // namespace mg

extern "C" mg_status mg_smoother_transpose(int32_t n, const double *A, const double *W, double *WT, void *stream)
{
    clear_error();
    if (n < 1 || n > 16383) return set_error(MG_ERR_ARG, "n = %d out of range", n);
    if (!A || !W || !WT) return set_error(MG_ERR_ARG, "null pointer");
    if (W == WT) return set_error(MG_ERR_ARG, "W and WT must not be the same buffer");
    MG_TRY(require_device());
    launch_al_transpose(n, A, W, WT, (hipStream_t)stream);
    MG_HIP(hipGetLastError());
    return MG_OK;
}

extern "C" mg_status mg_alpha_step(mg_ctx top, mg_ctx coarse, mg_ctx coarse_t, mg_net net, const mg_alpha_batch *b,
                                   const mg_train_opts *o_in, double *loss, double *losses, float *grad)
{
    clear_error();
    if (!top || !coarse || !coarse_t || !net || !b) return set_error(MG_ERR_ARG, "null argument");
    mg_train_opts o;
    if (o_in)
        o = *o_in;
    else
        mg_train_opts_default(&o);
    MG_TRY(check_train_opts(o));
    if (o.precision != 0) return set_error(MG_ERR_ARG, "the Algorithm 2 step trains in precision 0 (FP32)");
    mg_ctx_s &c = *top;
    const int B = c.nprob;
    if (c.opt.precision != MG_PREC_FP64) return set_error(MG_ERR_ARG, "top must be an FP64 context");
    if (b->nprob != B) return set_error(MG_ERR_SHAPE, "batch has %d problems, top %d", b->nprob, B);
    if (!b->k || !b->f || !b->u0 || !b->u_star) return set_error(MG_ERR_ARG, "batch arrays must be non-null");
    const int n = c.probs[0].n;
    int kmax = 0;
    for (int p = 0; p < B; ++p) {
        if (c.probs[p].n != n) return set_error(MG_ERR_SHAPE, "every problem of top must have the same n");
        if (b->k[p] < 1 || b->k[p] > kMaxCycles)
            return set_error(MG_ERR_ARG, "k[%d] = %d must be in [1, %d]", p, b->k[p], kMaxCycles);
        if (!b->f[p] || !b->u0[p] || !b->u_star[p] || (b->dW && !b->dW[p]))
            return set_error(MG_ERR_ARG, "problem %d: null vector", p);
        kmax = std::max(kmax, b->k[p]);
    }
    if (c.probs[0].nlev < 2) return set_error(MG_ERR_SHAPE, "top needs a coarser level (n > coarsest_n)");
    MG_TRY(check_alpha_coarse(c, *coarse, "coarse"));
    MG_TRY(check_alpha_coarse(c, *coarse_t, "coarse_t"));
    if (coarse == top || coarse_t == top) return set_error(MG_ERR_ARG, "the coarse contexts must differ from top");

    const LevelBuf &L0 = c.probs[0].lev[0];
    const int P = L0.P;
    const int64_t plane = L0.plane, vs = (plane + 31) / 32 * 32;
    const Work need = carve(nullptr, B, kmax, n, vs, plane);
    if (need.bytes > c.al_bytes) {
        MG_TRY(c.arena.alloc(&c.al_ws, need.bytes));
        c.al_bytes = need.bytes;
    }
    const Work w = carve((char *)c.al_ws, B, kmax, n, vs, plane);

    // the coarse contexts' slot tables are rewritten synchronously: their streams must be idle
    MG_HIP(hipStreamSynchronize(coarse->join.internal));
    MG_HIP(hipStreamSynchronize(coarse_t->join.internal));
    MG_TRY(ctx_set_live(*coarse, std::vector<char>(B, 1)));
    MG_TRY(ctx_set_live(*coarse_t, std::vector<char>(B, 1)));
    MG_TRY(c.join.enter());
    hipStream_t st = c.join.internal;
    MG_HIP(hipStreamSynchronize(st));  // the previous step's table upload has been read

    // small tables: problems, active masks per cycle, FP64 gradient outputs
    std::vector<AlphaProb> probs(B);
    std::vector<int> active((size_t)kmax * B);
    std::vector<double *> w64(B, nullptr);
    for (int p = 0; p < B; ++p) {
        AlphaProb &a = probs[p];
        a.A = c.probs[p].lev[0].A64;
        a.H = (const double *)c.probs[p].lev[0].H;
        const mg_ctx_s *cc[2] = {coarse, coarse_t};
        for (int q = 0; q < 2; ++q) {
            a.rc[q] = (double *)cc[q]->probs[p].lev[0].r;
            a.uc[q] = cc[q]->probs[p].u;
        }
        for (int i = 0; i < kmax; ++i) active[(size_t)i * B + p] = i < b->k[p];
        if (b->dW) w64[p] = b->dW[p];
    }
    const size_t sz_probs = sizeof(AlphaProb) * B, sz_act = sizeof(int) * active.size(),
                 sz_w64 = sizeof(double *) * B;
    c.al_host.resize(sz_probs + sz_act + sz_w64);
    std::memcpy(c.al_host.data(), probs.data(), sz_probs);
    std::memcpy(c.al_host.data() + sz_probs, active.data(), sz_act);
    std::memcpy(c.al_host.data() + sz_probs + sz_act, w64.data(), sz_w64);
    MG_HIP(hipMemcpyAsync(w.probs, c.al_host.data(), sz_probs, hipMemcpyHostToDevice, st));
    MG_HIP(hipMemcpyAsync(w.active, c.al_host.data() + sz_probs, sz_act, hipMemcpyHostToDevice, st));
    MG_HIP(hipMemcpyAsync(w.w64, c.al_host.data() + sz_probs + sz_act, sz_w64, hipMemcpyHostToDevice, st));

    // the trained level's smoother from the current parameters (FP64 inference)
    MG_TRY(ctx_infer(c, net, n, st, nullptr));

    auto V = [&](int k) { return w.vec + (int64_t)k * B * vs; };
    auto Rv = [&](int i) { return V(kNumVec + i); };
    auto Qv = [&](int i) { return V(kNumVec + kmax + i); };
    const int64_t nn = (int64_t)n * n;
    for (int p = 0; p < B; ++p) {
        launch_copy_field(n, 1, b->u0[p], n, nn, V(kU) + p * vs, P, plane, st);
        launch_copy_field(n, 1, b->f[p], n, nn, V(kF) + p * vs, P, plane, st);
        launch_copy_field(n, 1, b->u_star[p], n, nn, V(kUs) + p * vs, P, plane, st);
    }
    // one coarse cycle on every problem of a coarse context: u_c (cleared by the restriction) += V(r_c)
    auto coarse_cycle = [&](mg_ctx_s &cc) {
        launch_activate(cc.d_state, cc.nprob, st);
        ctx_enqueue_cycle(cc, st);
    };

    // ---- forward
    for (int i = 0; i < kmax; ++i) {
        const int *act = w.active + (size_t)i * B;
        double *r = Rv(i), *q = Qv(i);
        launch_al_apply_A(w.probs, B, n, P, plane, vs, V(kU), V(kF), -1.0, r, act, st);        // r = f - A u
        launch_al_H(w.probs, B, n, P, plane, vs, r, V(kA), false, false, act, st);              // a = H r
        launch_al_apply_A(w.probs, B, n, P, plane, vs, V(kA), r, -1.0, V(kS), act, st);        // s = r - A a
        launch_al_restrict(w.probs, 0, B, n, P, vs, V(kS), act, st);                             // r_c = R s
        coarse_cycle(*coarse);                                                                   // u_c = Psi_c(r_c)
        launch_al_prolong(w.probs, 0, B, n, P, vs, V(kA), V(kT), act, st);                     // t = a + P u_c
        launch_al_apply_A(w.probs, B, n, P, plane, vs, V(kT), r, -1.0, q, act, st);            // q = r - A t
        launch_al_axpy(B, n, P, vs, V(kU), 1.0, V(kT), V(kU), act, st);                         // u += t
        launch_al_H(w.probs, B, n, P, plane, vs, q, V(kU), false, true, act, st);               // u += H q
    }
    launch_al_dist(B, n, P, vs, V(kU), V(kUs), w.dist, st);
    std::vector<double> dist(B);
    MG_HIP(hipMemcpyAsync(dist.data(), w.dist, sizeof(double) * B, hipMemcpyDeviceToHost, st));
    MG_HIP(hipGetLastError());
    MG_HIP(hipStreamSynchronize(st));
    double total = 0.0;
    for (int p = 0; p < B; ++p) {
        if (!std::isfinite(dist[p])) {
            set_error(MG_ERR_DIVERGED, "problem %d: the loss is not finite (parameters left unchanged)", p);
            (void)c.join.leave();
            return MG_ERR_DIVERGED;
        }
        total += dist[p];
    }

    // ---- adjoint: lam = dL/du_k, then back through the cycles
    launch_al_seed(B, n, P, plane, vs, V(kU), V(kUs), w.dist, 1.0 / B, V(kLam), w.dH, st);
    for (int i = kmax - 1; i >= 0; --i) {
        const int *act = w.active + (size_t)i * B;
        const double *r = Rv(i), *q = Qv(i);
        launch_al_H(w.probs, B, n, P, plane, vs, V(kLam), V(kDq), true, false, act, st);       // dq = H^T lam
        launch_al_outer(B, n, P, plane, vs, V(kLam), q, w.dH, act, st);                         // dH += lam q^T
        launch_al_apply_A(w.probs, B, n, P, plane, vs, V(kDq), V(kLam), -1.0, V(kDt), act, st); // dt = lam - A dq
        launch_al_restrict(w.probs, 1, B, n, P, vs, V(kDt), act, st);                            // r_c = R dt
        coarse_cycle(*coarse_t);                                                                 // u_c = Psi_c^T(r_c)
        launch_al_prolong(w.probs, 1, B, n, P, vs, nullptr, V(kDs), act, st);                   // ds = P u_c
        launch_al_apply_A(w.probs, B, n, P, plane, vs, V(kDs), V(kDt), -1.0, V(kDa), act, st);  // da = dt - A ds
        launch_al_outer(B, n, P, plane, vs, V(kDa), r, w.dH, act, st);                          // dH += da r^T
        launch_al_axpy(B, n, P, vs, V(kDs), 1.0, V(kDq), V(kDr), act, st);                      // dr = ds + dq
        launch_al_H(w.probs, B, n, P, plane, vs, V(kDa), V(kDr), true, true, act, st);          // dr += H^T da
        launch_al_apply_A(w.probs, B, n, P, plane, vs, V(kDr), V(kLam), -1.0, V(kLam), act, st); // lam -= A dr
    }
    launch_al_dw(w.probs, B, n, P, plane, w.dH, b->dW ? w.w64 : nullptr, w.dout, st);

    // ---- network backward for dL/dW, then Adam
    std::vector<int> ns(B, n);
    std::vector<const double *> sten(B);
    std::vector<const float *> dout(B);
    for (int p = 0; p < B; ++p) {
        double *d = w.dense_A + (size_t)p * 9 * nn;
        launch_copy_field(n, 9, c.probs[p].lev[0].A64, P, plane, d, n, nn, st);
        sten[p] = d;
        dout[p] = w.dout + (size_t)p * 25 * nn;
    }
    MG_HIP(hipGetLastError());
    MG_TRY(net_backward_ext(*net, B, ns.data(), sten.data(), dout.data(), st));
    if (o.apply_update) net_adam(*net, o, st);
    if (grad) MG_HIP(hipMemcpyAsync(grad, net->grad, sizeof(float) * net->np, hipMemcpyDeviceToHost, st));
    MG_HIP(hipGetLastError());
    MG_HIP(hipStreamSynchronize(st));
    // later work of the network (its own stream) follows this step
    MG_HIP(hipEventRecord(net->join.ev, st));
    MG_HIP(hipStreamWaitEvent(net->join.internal, net->join.ev, 0));

    if (losses) std::copy(dist.begin(), dist.end(), losses);
    if (loss) *loss = total / B;
    return c.join.leave();
}
