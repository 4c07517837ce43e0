// Solver context: hierarchy set-up (Galerkin levels, coarsest inverse), the
// V-cycle schedule over size classes, the stationary solver with per-problem
// convergence masks, HIP-graph capture of one solver iteration, and smoother
// inference.
//
// Batching: all problems of a context are advanced together.  Every distinct
// level size forms a size class; each kernel launch covers every (problem,
// level) pair of one class (blockIdx.z selects the pair), so the number of
// launches per iteration depends on the number of distinct sizes, not on the
// number of problems.  A problem that has converged (or hit maxit) is masked
// out on the device, so one captured graph serves every iteration.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <string>

#include "internal.hpp"
#include "launch.hpp"
#include "stack.hpp"

using namespace mg;

namespace {

bool is_pow2m1(int n) { return n >= 1 && ((n + 1) & n) == 0; }

size_t tsize(const mg_ctx_s &c) { return c.opt.precision == MG_PREC_FP64 ? sizeof(double) : sizeof(float); }
size_t hsize(const mg_ctx_s &c) { return c.opt.precision == MG_PREC_FP64 ? sizeof(double) : sizeof(bf16_t); }

template <typename T>
const T *stencil_of(const LevelBuf &L);
template <>
const float *stencil_of<float>(const LevelBuf &L) { return L.A32; }
template <>
const double *stencil_of<double>(const LevelBuf &L) { return L.A64; }

template <typename S>
mg_status upload(Arena &arena, const std::vector<S> &v, void **dptr)
{
    MG_TRY(arena.alloc(dptr, sizeof(S) * v.size()));
    MG_HIP(hipMemcpy(*dptr, v.data(), sizeof(S) * v.size(), hipMemcpyHostToDevice));
    return MG_OK;
}

// A size class's slot table: uploaded, kept on the host for compaction, and
// room for the compacted copy.
template <typename S>
mg_status upload_class(Arena &arena, const std::vector<S> &v, const std::vector<int> &probs, SizeClass &sc)
{
    sc.nslots = (int)v.size();
    sc.probs = probs;
    sc.slot_bytes = sizeof(S);
    sc.host_slots.assign((const char *)v.data(), (const char *)(v.data() + v.size()));
    MG_TRY(upload(arena, v, &sc.d_slots));
    MG_TRY(arena.alloc(&sc.d_live, sizeof(S) * v.size()));
    sc.d_run = sc.d_slots;
    sc.nrun = sc.nslots;
    sc.run_slots.resize(sc.nslots);
    for (int s = 0; s < sc.nslots; ++s) sc.run_slots[s] = s;
    sc.live = sc.nslots > 0;
    return MG_OK;
}

// Builds the slot tables of every size class for compute type T.
template <typename T>
mg_status build_slots(mg_ctx_s &c)
{
    typedef typename SmootherStore<T>::type HT;
    std::map<int, std::vector<CycleSlot<T>>, std::greater<int>> cls;
    std::map<int, std::vector<OuterSlot<T>>, std::greater<int>> out;
    std::map<int, std::vector<int>> cls_probs, out_probs;
    std::vector<BottomSlot<T>> bottom;
    c.bottom_top_n = 0;
    for (int p = 0; p < c.nprob; ++p) {
        ProbBuf &pb = c.probs[p];
        int top = 0;  // first level handled by the bottom kernel
        while (pb.lev[top].n > kBottomMax) ++top;
        for (int l = 0; l < top; ++l) {
            const LevelBuf &L = pb.lev[l], &Lc = pb.lev[l + 1];
            CycleSlot<T> s{};
            s.prob = p;
            s.n = L.n;
            s.P = L.P;
            s.plane = L.plane;
            s.A = stencil_of<T>(L);
            s.sym = L.sym;
            // with the stack smoother, H points to the level's 54 weights (type T)
            s.H = c.opt.smoother == MG_SMOOTHER_STACK ? (const HT *)L.phi : (const HT *)L.H;
            s.r = (T *)L.r;
            s.e = (T *)L.e;
            s.s = (T *)L.s;
            s.rc = (T *)Lc.r;
            // the fused ascent of a level writes its post-smoothed correction to s (its
            // neighbours still read the pre-smoothed e in their halos); the bottom-levels
            // kernel leaves its top level's correction in e
            s.ec = (c.fused && l + 1 < top) ? (T *)Lc.s : (T *)Lc.e;
            s.nc = Lc.n;
            s.Pc = Lc.P;
            s.u = (c.fused && l == 0) ? pb.u : nullptr;
            cls[L.n].push_back(s);
            cls_probs[L.n].push_back(p);
        }
        const LevelBuf &L0 = pb.lev[0], &Lm = pb.lev[pb.nlev - 1];
        OuterSlot<T> o{};
        o.prob = p;
        o.n = L0.n;
        o.P = L0.P;
        o.plane = L0.plane;
        o.A64 = L0.A64;
        o.u = pb.u;
        o.f = pb.f;
        o.r = (T *)L0.r;
        o.e = (const T *)L0.e;
        o.partial = pb.partial;
        o.sym = pb.sym;
        out[L0.n].push_back(o);
        out_probs[L0.n].push_back(p);
        (void)Lm;
        BottomSlot<T> b{};
        b.prob = p;
        b.nlev = pb.nlev - top;
        for (int l = top; l < pb.nlev; ++l) {
            BottomLevel<T> &bl = b.lev[l - top];
            bl.n = pb.lev[l].n;
            bl.P = pb.lev[l].P;
            bl.plane = pb.lev[l].plane;
            bl.A = stencil_of<T>(pb.lev[l]);
            bl.H = c.opt.smoother == MG_SMOOTHER_STACK ? (const HT *)pb.lev[l].phi : (const HT *)pb.lev[l].H;
        }
        b.Ainv = pb.Ainv;
        b.r_in = (const T *)pb.lev[top].r;
        b.e_out = (T *)pb.lev[top].e;
        b.u = (c.fused && top == 0) ? pb.u : nullptr;
        b.partial = pb.partial;
        bottom.push_back(b);
        c.bottom_top_n = std::max(c.bottom_top_n, pb.lev[top].n);
    }
    for (auto &kv : cls) {
        SizeClass sc;
        sc.n = kv.first;
        MG_TRY(upload_class(c.arena, kv.second, cls_probs[kv.first], sc));
        c.classes.push_back(sc);
    }
    for (auto &kv : out) {
        SizeClass sc;
        sc.n = kv.first;
        MG_TRY(upload_class(c.arena, kv.second, out_probs[kv.first], sc));
        c.outer.push_back(sc);
    }
    std::vector<int> all(c.nprob);
    for (int p = 0; p < c.nprob; ++p) all[p] = p;
    c.bottom.n = c.bottom_top_n;
    MG_TRY(upload_class(c.arena, bottom, all, c.bottom));
    prepare_bottom<T>();
    if (c.opt.smoother == MG_SMOOTHER_STACK) prepare_stack_bottom<T>();
    return MG_OK;
}

// One V-cycle e = V(r) on every active problem (Algorithm 1, correction form).
// V(1,1) runs the fused level kernels (descend, bottom, ascend), which add
// the finest correction to u themselves; other sweep counts run the
// step-by-step kernels and leave u += e to enqueue_update.  check: the fused
// bottom kernel (network, Jacobi or stack smoother) also applies the stopping
// rule (see enqueue_iteration).
template <typename T>
void enqueue_vcycle(mg_ctx_s &c, hipStream_t st, const SolveParams *check = nullptr)
{
    const bool cnn = c.opt.smoother == MG_SMOOTHER_CNN, stack = c.opt.smoother == MG_SMOOTHER_STACK;
    const double w = c.opt.omega;
    auto smooth = [&](const CycleSlot<T> *s, const SizeClass &k, bool first, bool post = false) {
        if (stack)
            launch_stack_cycle<T>(s, k.nrun, k.n, first ? kStackFirst : post ? kStackPost : kStackPre, c.d_state,
                                  st);
        else if (first)
            launch_smooth_first<T>(s, k.nrun, k.n, cnn, w, c.d_state, st);
        else
            launch_smooth_apply<T>(s, k.nrun, k.n, cnn, w, c.d_state, st);
    };
    if (c.fused && stack) {
        for (const SizeClass &k : c.classes)  // descending sizes
            if (k.live) launch_stack_descend<T>((const CycleSlot<T> *)k.d_run, k.nrun, (k.n - 1) / 2, c.d_state, st);
        if (c.bottom.live)
            launch_stack_bottom<T>((const BottomSlot<T> *)c.bottom.d_run, c.bottom.nrun, c.bottom_top_n, 1, 1,
                                   c.d_state, check, st);
        for (auto it = c.classes.rbegin(); it != c.classes.rend(); ++it)  // ascending sizes
            if (it->live) launch_stack_ascend<T>((const CycleSlot<T> *)it->d_run, it->nrun, it->n, c.d_state, st);
        return;
    }
    if (c.fused) {
        for (const SizeClass &k : c.classes)  // descending sizes
            if (k.live)
                launch_descend<T>((const CycleSlot<T> *)k.d_run, k.nrun, k.n, cnn, w, c.d_state, st, k.tile[0]);
        if (c.bottom.live)
            launch_bottom<T>((const BottomSlot<T> *)c.bottom.d_run, c.bottom.nrun, c.bottom_top_n, cnn, w, 1, 1,
                             c.d_state, check, st);
        for (auto it = c.classes.rbegin(); it != c.classes.rend(); ++it)  // ascending sizes
            if (it->live)
                launch_ascend<T>((const CycleSlot<T> *)it->d_run, it->nrun, it->n, cnn, w, c.d_state, st,
                                 it->tile[1]);
        return;
    }
    for (const SizeClass &k : c.classes) {  // descending sizes
        if (!k.live) continue;
        auto *s = (const CycleSlot<T> *)k.d_run;
        if (c.opt.nu_pre == 0) {
            launch_zero_e<T>(s, k.nrun, k.n, c.d_state, st);
        } else {
            smooth(s, k, true);
            for (int it = 1; it < c.opt.nu_pre; ++it) {
                launch_residual<T>(s, k.nrun, k.n, c.d_state, st);
                smooth(s, k, false);
            }
        }
        launch_residual_restrict<T>(s, k.nrun, k.n, c.d_state, st);
    }
    if (c.bottom.live) {
        if (stack)
            launch_stack_bottom<T>((const BottomSlot<T> *)c.bottom.d_run, c.bottom.nrun, c.bottom_top_n, c.opt.nu_pre,
                                   c.opt.nu_post, c.d_state, nullptr, st);
        else
            launch_bottom<T>((const BottomSlot<T> *)c.bottom.d_run, c.bottom.nrun, c.bottom_top_n, cnn, w,
                             c.opt.nu_pre, c.opt.nu_post, c.d_state, nullptr, st);
    }
    for (auto it = c.classes.rbegin(); it != c.classes.rend(); ++it) {  // ascending sizes
        const SizeClass &k = *it;
        if (!k.live) continue;
        auto *s = (const CycleSlot<T> *)k.d_run;
        launch_prolong<T>(s, k.nrun, k.n, c.d_state, st);
        for (int q = 0; q < c.opt.nu_post; ++q) {
            launch_residual<T>(s, k.nrun, k.n, c.d_state, st);
            smooth(s, k, false, true);
        }
    }
}

template <typename T>
void enqueue_outer_residual(mg_ctx_s &c, hipStream_t st)
{
    for (const SizeClass &k : c.outer)
        if (k.live) launch_outer_residual<T>((const OuterSlot<T> *)k.d_run, k.nrun, k.n, c.d_state, st);
}

template <typename T>
void enqueue_check(mg_ctx_s &c, int init, hipStream_t st)
{
    for (const SizeClass &k : c.outer)
        if (k.live) launch_check<T>((const OuterSlot<T> *)k.d_run, k.nrun, c.d_state, c.d_params, init, st);
}

// u += e where the V-cycle did not do it.
template <typename T>
void enqueue_update(mg_ctx_s &c, hipStream_t st)
{
    if (c.fused) return;
    for (const SizeClass &k : c.outer)
        if (k.live) launch_update_u<T>((const OuterSlot<T> *)k.d_run, k.nrun, k.n, c.d_state, st);
}

// One solver iteration: residual and stopping rule, V-cycle, update.  The
// fused V(1,1) cycle applies the rule in its bottom kernel (one workgroup per
// problem, which has the time to sum the residual's block sums while its own
// loads arrive): one launch fewer per iteration.  The descent has then
// already run on a residual that may meet the tolerance; only the ascent and
// u depend on the rule, and they follow it.
// (A completion counter shared by every block of the residual kernel, to apply
// the rule there instead, serialises thousands of atomics and costs more than
// a launch.)
template <typename T>
void enqueue_iteration(mg_ctx_s &c, hipStream_t st)
{
    const bool folded = c.fused;
    enqueue_outer_residual<T>(c, st);
    if (!folded) enqueue_check<T>(c, 0, st);
    enqueue_vcycle<T>(c, st, folded ? c.d_params : nullptr);
    enqueue_update<T>(c, st);
}

void enqueue_iteration_any(mg_ctx_s &c, hipStream_t st)
{
    if (c.opt.precision == MG_PREC_FP64)
        enqueue_iteration<double>(c, st);
    else
        enqueue_iteration<float>(c, st);
}

mg_status validate_options(const mg_options &o)
{
    if (o.smoother != MG_SMOOTHER_JACOBI && o.smoother != MG_SMOOTHER_CNN && o.smoother != MG_SMOOTHER_STACK)
        return set_error(MG_ERR_ARG, "smoother must be MG_SMOOTHER_JACOBI, MG_SMOOTHER_CNN or MG_SMOOTHER_STACK");
    if (o.nu_pre < 0 || o.nu_pre > 8 || o.nu_post < 0 || o.nu_post > 8)
        return set_error(MG_ERR_ARG, "nu_pre and nu_post must be in [0, 8]");
    if (!(o.omega > 0.0 && o.omega < 2.0)) return set_error(MG_ERR_ARG, "omega must be in (0, 2)");
    if (o.coarsest_n != 1 && o.coarsest_n != 3 && o.coarsest_n != 7)
        return set_error(MG_ERR_ARG, "coarsest_n must be 1, 3 or 7");
    if (o.precision != MG_PREC_FP64 && o.precision != MG_PREC_MIXED)
        return set_error(MG_ERR_ARG, "precision must be MG_PREC_FP64 or MG_PREC_MIXED");
    if (o.check_every < 0) return set_error(MG_ERR_ARG, "check_every must be >= 0");
    if (o.fallback != 0 && o.fallback != 1) return set_error(MG_ERR_ARG, "fallback must be 0 or 1");
    if (o.fallback && o.smoother == MG_SMOOTHER_STACK)
        return set_error(MG_ERR_ARG, "the fallback to damped Jacobi applies to the CNN smoother only");
    return MG_OK;
}

void destroy_ctx(mg_ctx c)
{
    if (!c) return;
    if (c->join.internal) (void)hipStreamSynchronize(c->join.internal);
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->t0) (void)hipEventDestroy(c->t0);
    if (c->t1) (void)hipEventDestroy(c->t1);
    for (hipEvent_t e : c->ev_state)
        if (e) (void)hipEventDestroy(e);
    if (c->h_state) (void)hipHostFree(c->h_state);
    c->arena.release();
    c->join.destroy();
    delete c;
}

// Finest stencil into the pitched layout (checked; its FP32 copy and symmetry
// flags in the same pass), the Galerkin levels in FP64, their FP32 copies and
// symmetry flags, and the coarsest inverse.
void rebuild_problem(mg_ctx_s &c, int p, const double *stencil, hipStream_t st)
{
    ProbBuf &pb = c.probs[p];
    const LevelBuf &L0 = pb.lev[0];
    const bool mixed = c.opt.precision == MG_PREC_MIXED;
    // level 0 in one pass over the caller's stencil: copies, checks, both symmetry flags
    launch_ingest(pb.n, stencil, L0.P, L0.plane, L0.A64, mixed ? L0.A32 : nullptr, c.d_flag, pb.sym, L0.sym, st);
    for (int q = 0; q + 1 < pb.nlev; ++q) {
        const LevelBuf &F = pb.lev[q], &Cc = pb.lev[q + 1];
        launch_galerkin(F.n, F.P, F.plane, F.A64, Cc.P, Cc.plane, Cc.A64, st);
    }
    for (int q = 1; q < pb.nlev; ++q) {
        const LevelBuf &L = pb.lev[q];
        if (c.opt.precision == MG_PREC_MIXED) {
            launch_to_f32(9 * L.plane, L.A64, L.A32, st);
            launch_check_symmetric(L.n, L.P, L.plane, L.A32, L.sym, st);
        } else {
            launch_check_symmetric(L.n, L.P, L.plane, L.A64, L.sym, st);
        }
    }
    const LevelBuf &Lm = pb.lev[pb.nlev - 1];
    launch_coarse_factor(Lm.n, Lm.P, Lm.plane, Lm.A64, pb.Ainv, c.d_flag, st);
}

mg_status read_flag(mg_ctx_s &c, hipStream_t st)
{
    MG_HIP(hipStreamSynchronize(st));
    int flag = 0;
    MG_HIP(hipMemcpy(&flag, c.d_flag, sizeof(int), hipMemcpyDeviceToHost));
    if (flag & 1) return set_error(MG_ERR_ARG, "a stencil entry couples to a node outside the grid");
    if (flag & 2) return set_error(MG_ERR_ARG, "a stencil centre entry is not positive");
    if (flag & 4) return set_error(MG_ERR_ARG, "a stencil entry is not finite");
    if (flag & 8) return set_error(MG_ERR_ARG, "the coarsest-level matrix is not positive definite");
    return MG_OK;
}

// The level table of the one-launch MFMA inference: every level above the
// coarsest of every problem, by size (largest first) and problem.
mg_status build_cnn_table(mg_ctx_s &c)
{
    std::vector<CnnLevelDesc> t;
    for (const ProbBuf &pb : c.probs)
        for (int l = 0; l + 1 < pb.nlev; ++l) {
            const LevelBuf &L = pb.lev[l];
            t.push_back(CnnLevelDesc{L.n, L.P, L.plane, L.A32, (bf16_t *)L.H, 0});
        }
    std::stable_sort(t.begin(), t.end(), [](const CnnLevelDesc &a, const CnnLevelDesc &b) { return a.n > b.n; });
    int tiles = 0;
    for (CnnLevelDesc &d : t) {
        d.tile0 = tiles;
        tiles += cnn_level_tiles(d.n);
    }
    c.n_cnn_levels = (int)t.size();
    c.cnn_tiles = tiles;
    if (t.empty()) return MG_OK;
    return upload(c.arena, t, (void **)&c.d_cnn_levels);
}

mg_status setup_impl(mg_ctx_s &c, const mg_problem *probs, hipStream_t user)
{
    MG_TRY(c.join.init(user));
    c.arena.stream = c.join.internal;
    MG_HIP(hipEventCreate(&c.t0));
    MG_HIP(hipEventCreate(&c.t1));
    for (hipEvent_t &e : c.ev_state) MG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    MG_HIP(hipHostMalloc((void **)&c.h_state, 2 * sizeof(SolveState) * c.nprob, hipHostMallocDefault));
    MG_TRY(c.join.enter());
    hipStream_t st = c.join.internal;
    const bool mixed = c.opt.precision == MG_PREC_MIXED;
    c.probs.resize(c.nprob);
    MG_TRY(c.arena.alloc((void **)&c.d_flag, sizeof(int)));
    for (int p = 0; p < c.nprob; ++p) {
        ProbBuf &pb = c.probs[p];
        pb.n = probs[p].n;
        int m = pb.n, l = 0;
        for (;;) {
            LevelBuf &L = pb.lev[l];
            L.n = m;
            L.P = m + 1;
            L.plane = plane_of(L.n, L.P);
            const size_t v = (size_t)L.plane;
            MG_TRY(c.arena.alloc((void **)&L.A64, 9 * v * sizeof(double)));
            if (mixed) MG_TRY(c.arena.alloc((void **)&L.A32, 9 * v * sizeof(float)));
            MG_TRY(c.arena.alloc(&L.r, v * tsize(c)));
            MG_TRY(c.arena.alloc(&L.e, v * tsize(c)));
            MG_TRY(c.arena.alloc((void **)&L.sym, sizeof(int)));
            ++l;
            if (m == c.opt.coarsest_n) break;
            MG_TRY(c.arena.alloc(&L.H, kSmoother * v * hsize(c)));
            if (c.opt.smoother == MG_SMOOTHER_STACK) MG_TRY(c.arena.alloc(&L.phi, 2 * kStackWeights * tsize(c)));
            MG_TRY(c.arena.alloc(&L.s, v * tsize(c)));
            m = (m - 1) / 2;
        }
        pb.nlev = l;
        const LevelBuf &L0 = pb.lev[0];
        MG_TRY(c.arena.alloc((void **)&pb.u, (size_t)L0.plane * sizeof(double)));
        MG_TRY(c.arena.alloc((void **)&pb.f, (size_t)L0.plane * sizeof(double)));
        const int mm = c.opt.coarsest_n * c.opt.coarsest_n;
        MG_TRY(c.arena.alloc((void **)&pb.Ainv, (size_t)mm * mm * sizeof(double)));
        pb.nparts = outer_residual_parts(pb.n);
        MG_TRY(c.arena.alloc((void **)&pb.partial, (size_t)pb.nparts * sizeof(double)));
        MG_TRY(c.arena.alloc((void **)&pb.sym, sizeof(int)));
        rebuild_problem(c, p, probs[p].stencil, st);
        MG_HIP(hipGetLastError());
    }
    if (mixed) {
        MG_TRY(build_slots<float>(c));
        MG_TRY(build_cnn_table(c));
    } else {
        MG_TRY(build_slots<double>(c));
    }
    std::vector<SolveState> init(c.nprob);
    for (int p = 0; p < c.nprob; ++p) {
        std::memset(&init[p], 0, sizeof(SolveState));
        init[p].nparts = c.probs[p].nparts;
    }
    MG_TRY(upload(c.arena, init, (void **)&c.d_state));
    MG_TRY(c.arena.alloc((void **)&c.d_params, sizeof(SolveParams)));
    MG_TRY(c.arena.alloc((void **)&c.d_scalar, sizeof(double)));
    MG_TRY(read_flag(c, st));
    MG_TRY(c.join.leave());
    return MG_OK;
}

mg_status check_ctx(mg_ctx c)
{
    if (!c) return set_error(MG_ERR_ARG, "context is null");
    return MG_OK;
}

mg_status check_level(mg_ctx c, int prob, int level, bool smoother)
{
    MG_TRY(check_ctx(c));
    if (prob < 0 || prob >= c->nprob) return set_error(MG_ERR_ARG, "problem index %d out of range", prob);
    if (smoother && c->opt.smoother == MG_SMOOTHER_STACK)
        return set_error(MG_ERR_STATE, "the stack smoother has no per-point field (mg_set_stack installs its weights)");
    const int top = c->probs[prob].nlev - (smoother ? 1 : 0);
    if (level < 0 || level >= top) return set_error(MG_ERR_ARG, "level %d out of range", level);
    return MG_OK;
}

mg_status check_vectors(mg_ctx c, const double *const *f, double *const *u)
{
    if (!f || !u) return set_error(MG_ERR_ARG, "f and u must be non-null arrays of device pointers");
    for (int p = 0; p < c->nprob; ++p)
        if (!f[p] || !u[p]) return set_error(MG_ERR_ARG, "f[%d] or u[%d] is null", p, p);
    return MG_OK;
}

void copy_in(mg_ctx_s &c, const double *const *f, double *const *u, bool zero_u, hipStream_t st)
{
    for (int p = 0; p < c.nprob; ++p) {
        const ProbBuf &pb = c.probs[p];
        const LevelBuf &L0 = pb.lev[0];
        launch_copy_field(pb.n, 1, f[p], pb.n, (int64_t)pb.n * pb.n, pb.f, L0.P, L0.plane, st);
        if (zero_u)
            launch_zero_f64(pb.u, L0.plane, st);
        else
            launch_copy_field(pb.n, 1, u[p], pb.n, (int64_t)pb.n * pb.n, pb.u, L0.P, L0.plane, st);
    }
}

void copy_out(mg_ctx_s &c, double *const *u, hipStream_t st)
{
    for (int p = 0; p < c.nprob; ++p) {
        const ProbBuf &pb = c.probs[p];
        const LevelBuf &L0 = pb.lev[0];
        launch_copy_field(pb.n, 1, pb.u, L0.P, L0.plane, u[p], pb.n, (int64_t)pb.n * pb.n, st);
    }
}

void drop_graph(mg_ctx_s &c)
{
    if (c.graph_exec) (void)hipGraphExecDestroy(c.graph_exec);
    if (c.graph) (void)hipGraphDestroy(c.graph);
    c.graph_exec = nullptr;
    c.graph = nullptr;
}

// Keeps the launches to the problems that still iterate: each size class
// launches a compacted copy of its slot table holding only the active
// problems' slots (a class with none is left out), and the captured iteration
// is rebuilt whenever that changes.  Blocks of finished problems would return
// at once, but an uneven batch's last few slow problems would still pay for
// dispatching every finished problem's tiles of every level size.  Called with
// the stream idle (the slot copies are synchronous).
mg_status update_live(mg_ctx_s &c, const std::vector<char> &active)
{
    bool changed = false;
    auto compact = [&](SizeClass &k) -> mg_status {
        std::vector<int> idx;
        for (int s = 0; s < k.nslots; ++s)
            if (active[k.probs[s]]) idx.push_back(s);
        if (idx == k.run_slots) return MG_OK;
        changed = true;
        const int cnt = (int)idx.size();
        k.live = cnt > 0;
        k.run_slots = idx;
        k.nrun = cnt;
        if (cnt == k.nslots) {
            k.d_run = k.d_slots;
            return MG_OK;
        }
        std::vector<char> buf((size_t)cnt * k.slot_bytes);
        for (int q = 0; q < cnt; ++q)
            std::memcpy(&buf[(size_t)q * k.slot_bytes], &k.host_slots[(size_t)idx[q] * k.slot_bytes], k.slot_bytes);
        if (cnt > 0) MG_HIP(hipMemcpy(k.d_live, buf.data(), buf.size(), hipMemcpyHostToDevice));
        k.d_run = k.d_live;
        return MG_OK;
    };
    for (SizeClass &k : c.classes) MG_TRY(compact(k));
    for (SizeClass &k : c.outer) MG_TRY(compact(k));
    MG_TRY(compact(c.bottom));
    // the captured iteration no longer matches: mark it (ensure_graph rebuilds it before the next
    // replay) rather than destroy it here, so the calls that change the live set free nothing
    if (changed) c.graph_stale = true;
    return MG_OK;
}

mg_status ensure_graph(mg_ctx_s &c)
{
    if (c.graph_stale) {
        drop_graph(c);
        c.graph_stale = false;
    }
    if (c.graph_exec || !c.opt.use_graph) return MG_OK;
    hipStream_t st = c.join.internal;
    // one check block of iterations per graph: consecutive graph launches leave a gap of several
    // microseconds between them on the device, kernels inside one graph follow each other at once
    MG_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    for (int q = 0; q < c.opt.check_every; ++q) enqueue_iteration_any(c, st);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(st, &g);
    if (e != hipSuccess) return set_error(MG_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
    c.graph = g;
    MG_HIP(hipGraphInstantiate(&c.graph_exec, c.graph, nullptr, nullptr, 0));
    return MG_OK;
}

}  // namespace

// Services of the context for the Krylov driver (krylov.cpp).
namespace mg {
mg_status ctx_check(mg_ctx c) { return check_ctx(c); }
mg_status ctx_check_smoother(const mg_ctx_s &c)
{
    if (c.opt.smoother == MG_SMOOTHER_CNN && !c.smoother_ready)
        return set_error(MG_ERR_STATE, "CNN smoother requested but mg_smoother_infer has not run");
    if (c.opt.smoother == MG_SMOOTHER_STACK)
        for (int p = 0; p < c.nprob; ++p)
            for (int l = 0; l + 1 < c.probs[p].nlev; ++l)
                if (!c.probs[p].lev[l].phi_set)
                    return set_error(MG_ERR_STATE, "problem %d level %d: no stack smoother installed (mg_set_stack)",
                                     p, l);
    return MG_OK;
}
mg_status ctx_check_vectors(mg_ctx c, const double *const *f, double *const *u) { return check_vectors(c, f, u); }
mg_status ctx_set_live(mg_ctx_s &c, const std::vector<char> &active) { return update_live(c, active); }
void ctx_enqueue_cycle(mg_ctx_s &c, hipStream_t st)
{
    if (c.opt.precision == MG_PREC_FP64) {
        enqueue_vcycle<double>(c, st);
        enqueue_update<double>(c, st);
    } else {
        enqueue_vcycle<float>(c, st);
        enqueue_update<float>(c, st);
    }
}
}  // namespace mg

extern "C" {

mg_status mg_setup(const mg_problem *probs, int32_t nprob, const mg_options *opt_in, void *stream, mg_ctx *out)
{
    clear_error();
    if (!out) return set_error(MG_ERR_ARG, "out is null");
    *out = nullptr;
    if (!probs || nprob < 1) return set_error(MG_ERR_ARG, "need at least one problem");
    mg_options opt;
    if (opt_in)
        opt = *opt_in;
    else
        mg_options_default(&opt);
    if (opt.check_every == 0) opt.check_every = 16;
    MG_TRY(validate_options(opt));
    for (int p = 0; p < nprob; ++p) {
        const int n = probs[p].n;
        if (!is_pow2m1(n) || n < opt.coarsest_n || n > 8191)
            return set_error(MG_ERR_ARG, "problem %d: n = %d must be 2^k - 1 with coarsest_n <= n <= 8191", p, n);
        if (!probs[p].stencil) return set_error(MG_ERR_ARG, "problem %d: stencil is null", p);
        int levels = 1;
        for (int m = n; m > opt.coarsest_n; m = (m - 1) / 2) ++levels;
        if (levels > kMaxLevels) return set_error(MG_ERR_ARG, "problem %d: too many levels", p);
    }
    MG_TRY(require_device());
    mg_ctx c = new mg_ctx_s();
    c->opt = opt;
    c->fused = opt.nu_pre == 1 && opt.nu_post == 1;
    c->nprob = nprob;
    mg_status s = setup_impl(*c, probs, (hipStream_t)stream);
    if (s < 0) {
        destroy_ctx(c);
        return s;
    }
    *out = c;
    return MG_OK;
}

mg_status mg_destroy(mg_ctx ctx)
{
    clear_error();
    destroy_ctx(ctx);
    return MG_OK;
}

mg_status mg_num_levels(mg_ctx ctx, int32_t prob, int32_t *nlev)
{
    clear_error();
    MG_TRY(check_ctx(ctx));
    if (!nlev) return set_error(MG_ERR_ARG, "nlev is null");
    if (prob < 0 || prob >= ctx->nprob) return set_error(MG_ERR_ARG, "problem index out of range");
    *nlev = ctx->probs[prob].nlev;
    return MG_OK;
}

mg_status mg_get_stencil(mg_ctx ctx, int32_t prob, int32_t level, double *out)
{
    clear_error();
    MG_TRY(check_level(ctx, prob, level, false));
    if (!out) return set_error(MG_ERR_ARG, "out is null");
    const LevelBuf &L = ctx->probs[prob].lev[level];
    MG_TRY(ctx->join.enter());
    launch_copy_field(L.n, 9, L.A64, L.P, L.plane, out, L.n, (int64_t)L.n * L.n, ctx->join.internal);
    MG_HIP(hipGetLastError());
    return ctx->join.leave();
}

mg_status mg_set_smoother(mg_ctx ctx, int32_t prob, int32_t level, const double *W)
{
    clear_error();
    MG_TRY(check_level(ctx, prob, level, true));
    if (!W) return set_error(MG_ERR_ARG, "W is null");
    const LevelBuf &L = ctx->probs[prob].lev[level];
    MG_TRY(ctx->join.enter());
    hipStream_t st = ctx->join.internal;
    if (ctx->opt.precision == MG_PREC_FP64)
        launch_set_smoother<double>(L.n, L.P, L.plane, W, L.n, (int64_t)L.n * L.n, L.A64, (double *)L.H, st);
    else
        launch_set_smoother<float>(L.n, L.P, L.plane, W, L.n, (int64_t)L.n * L.n, L.A64, (bf16_t *)L.H, st);
    MG_HIP(hipGetLastError());
    ctx->smoother_ready = true;
    return ctx->join.leave();
}

mg_status mg_get_smoother(mg_ctx ctx, int32_t prob, int32_t level, double *out)
{
    clear_error();
    MG_TRY(check_level(ctx, prob, level, true));
    if (!out) return set_error(MG_ERR_ARG, "out is null");
    const LevelBuf &L = ctx->probs[prob].lev[level];
    MG_TRY(ctx->join.enter());
    hipStream_t st = ctx->join.internal;
    if (ctx->opt.precision == MG_PREC_FP64)
        launch_get_smoother<double>(L.n, L.P, L.plane, (const double *)L.H, L.A64, out, L.n, (int64_t)L.n * L.n, st);
    else
        launch_get_smoother<float>(L.n, L.P, L.plane, (const bf16_t *)L.H, L.A64, out, L.n, (int64_t)L.n * L.n, st);
    MG_HIP(hipGetLastError());
    return ctx->join.leave();
}

mg_status mg_vcycle(mg_ctx ctx, const double *const *f, double *const *u)
{
    clear_error();
    MG_TRY(check_ctx(ctx));
    MG_TRY(check_vectors(ctx, f, u));
    MG_TRY(ctx_check_smoother(*ctx));
    MG_TRY(ctx->join.enter());
    hipStream_t st = ctx->join.internal;
    copy_in(*ctx, f, u, false, st);
    MG_TRY(update_live(*ctx, std::vector<char>(ctx->nprob, 1)));  // every problem takes part
    launch_activate(ctx->d_state, ctx->nprob, st);
    if (ctx->opt.precision == MG_PREC_FP64) {
        enqueue_outer_residual<double>(*ctx, st);
        enqueue_vcycle<double>(*ctx, st);
        enqueue_update<double>(*ctx, st);
    } else {
        enqueue_outer_residual<float>(*ctx, st);
        enqueue_vcycle<float>(*ctx, st);
        enqueue_update<float>(*ctx, st);
    }
    copy_out(*ctx, u, st);
    MG_HIP(hipGetLastError());
    return ctx->join.leave();
}

mg_status mg_solve(mg_ctx ctx, const double *const *f, double *const *u, double rtol, int32_t maxit, int32_t *iters,
                   double *relres, int32_t *status, double *history)
{
    clear_error();
    MG_TRY(check_ctx(ctx));
    MG_TRY(check_vectors(ctx, f, u));
    if (!(rtol >= 0.0) || maxit < 0 || maxit > 100000000)
        return set_error(MG_ERR_ARG, "need rtol >= 0 and 0 <= maxit <= 1e8");
    MG_TRY(ctx_check_smoother(*ctx));
    mg_ctx_s &c = *ctx;
    const int stride = maxit + 1;
    if (history) {
        const size_t need = (size_t)c.nprob * stride;
        if (need > c.history_cap) {
            void *p = nullptr;
            MG_TRY(c.arena.alloc(&p, need * sizeof(double)));
            c.d_history = (double *)p;
            c.history_cap = need;
        }
    }
    MG_TRY(update_live(c, std::vector<char>(c.nprob, 1)));
    MG_TRY(c.join.enter());
    hipStream_t st = c.join.internal;
    MG_HIP(hipEventRecord(c.t0, st));
    copy_in(c, f, u, true, st);
    if (history) launch_zero_f64(c.d_history, (int64_t)c.nprob * stride, st);
    static thread_local SolveParams prm;
    prm.tol = rtol;
    prm.maxit = maxit;
    prm.hist_stride = stride;
    prm.history = history ? c.d_history : nullptr;
    prm.fallback = c.opt.fallback && c.opt.smoother == MG_SMOOTHER_CNN;
    c.fell_back.assign(c.nprob, 0);
    MG_HIP(hipMemcpyAsync(c.d_params, &prm, sizeof prm, hipMemcpyHostToDevice, st));
    // ||f||: the residual of u = 0
    launch_activate(c.d_state, c.nprob, st);
    if (c.opt.precision == MG_PREC_FP64) {
        enqueue_outer_residual<double>(c, st);
        enqueue_check<double>(c, 1, st);
    } else {
        enqueue_outer_residual<float>(c, st);
        enqueue_check<float>(c, 1, st);
    }
    std::vector<SolveState> hs(c.nprob);
    std::vector<char> act(c.nprob), live(c.nprob, 1);
    const int every = c.opt.check_every;
    int64_t replays = 0;
    // maxit cycles and the last check take maxit + 1 replays; a problem paused for the fallback
    // spends the rest of its check block without cycling, so each switch adds one block
    int64_t budget = (int64_t)maxit + 2;
    // One check block of iterations, then the problems' states copied to pinned host memory and an
    // event behind the copy.  Without the fallback the host only reads those states, so when some
    // problem is expected to iterate beyond the block in flight, the next block is queued before the
    // host waits for the last one's copy and the device does not idle while the host decides.  The
    // expectation: its relative residual after the last block, reduced once more by that block's
    // factor, still above 4 tol, and maxit not reached (a block queued behind the one that ends the
    // solve would run with every problem inactive: 1.5 ms at n = 4095).  A change of the live set
    // waits until the stream has drained, since it rewrites slot tables that a queued block reads.
    const bool ahead = !prm.fallback;
    std::vector<double> rel1(c.nprob, 0.0), rel2(c.nprob, 0.0);  // after the last two blocks read
    bool more = false;
    SolveState *const hbuf[2] = {c.h_state, c.h_state + c.nprob};
    int64_t rep[2] = {0, 0};
    auto enqueue_block = [&](int b) -> mg_status {
        MG_TRY(ensure_graph(c));  // (re)captured with the live classes; the stream is idle whenever it changes
        if (c.graph_exec)
            MG_HIP(hipGraphLaunch(c.graph_exec, st));  // every iterations
        else
            for (int q = 0; q < every; ++q) enqueue_iteration_any(c, st);
        replays += every;
        rep[b] = replays;
        MG_HIP(hipMemcpyAsync(hbuf[b], c.d_state, sizeof(SolveState) * c.nprob, hipMemcpyDeviceToHost, st));
        MG_HIP(hipEventRecord(c.ev_state[b], st));
        return MG_OK;
    };
    int cur = 0;
    MG_TRY(enqueue_block(cur));
    for (;;) {
        const int nxt = 1 - cur;
        const bool queued = ahead && more;
        if (queued) MG_TRY(enqueue_block(nxt));
        MG_HIP(hipEventSynchronize(c.ev_state[cur]));
        SolveState *const hsb = hbuf[cur];
        // problems paused by the fallback rule: damped Jacobi from now on (the stream is idle here)
        bool resumed = false;
        for (int p = 0; p < c.nprob && !ahead; ++p) {
            SolveState &s = hsb[p];
            if (s.status != 2 || (s.fallback != 1 && s.fallback != 3)) continue;
            const ProbBuf &pb = c.probs[p];
            for (int l = 0; l + 1 < pb.nlev; ++l) {
                const LevelBuf &L = pb.lev[l];
                if (c.opt.precision == MG_PREC_FP64)
                    launch_jacobi_smoother<double>(L.n, L.P, L.plane, L.A64, c.opt.omega, (double *)L.H, st);
                else
                    launch_jacobi_smoother<float>(L.n, L.P, L.plane, L.A64, c.opt.omega, (bf16_t *)L.H, st);
            }
            const bool restart = s.fallback == 3;  // after a divergence u is no starting point
            if (restart) launch_zero_f64(pb.u, pb.lev[0].plane, st);
            s.best = restart ? 1.0 : s.relres;
            s.stall = 0;
            s.fallback = 2;
            s.status = 0;
            s.active = 1;
            c.fell_back[p] = 1;
            resumed = true;
        }
        if (resumed) {
            MG_HIP(hipMemcpyAsync(c.d_state, hsb, sizeof(SolveState) * c.nprob, hipMemcpyHostToDevice, st));
            MG_HIP(hipStreamSynchronize(st));
            budget += every;
        }
        bool any = false;
        for (int p = 0; p < c.nprob; ++p) {
            act[p] = hsb[p].active != 0;
            any |= act[p] != 0;
        }
        if (!any || rep[cur] > budget) break;
        more = false;
        for (int p = 0; p < c.nprob; ++p) {
            rel2[p] = rel1[p];
            rel1[p] = hsb[p].relres;
            if (act[p] && rel2[p] > 0.0 && (int64_t)hsb[p].iters + every < maxit &&
                rel1[p] * (rel1[p] / rel2[p]) > 4.0 * rtol)
                more = true;
        }
        if (act != live) {
            if (queued) MG_HIP(hipStreamSynchronize(st));
            MG_TRY(update_live(c, act));
            live = act;
        }
        if (!queued) MG_TRY(enqueue_block(nxt));
        cur = nxt;
    }
    copy_out(c, u, st);
    MG_HIP(hipEventRecord(c.t1, st));
    MG_HIP(hipGetLastError());
    MG_HIP(hipStreamSynchronize(st));
    float ms = 0.0f;
    MG_HIP(hipEventElapsedTime(&ms, c.t0, c.t1));
    c.last_ms = ms;
    MG_HIP(hipMemcpy(hs.data(), c.d_state, sizeof(SolveState) * c.nprob, hipMemcpyDeviceToHost));
    if (history) MG_HIP(hipMemcpy(history, c.d_history, sizeof(double) * c.nprob * stride, hipMemcpyDeviceToHost));
    mg_status agg = MG_OK;
    for (int p = 0; p < c.nprob; ++p)
        if (c.fell_back[p]) c.smoother_ready = false;  // the learned smoother was overwritten
    for (int p = 0; p < c.nprob; ++p) {
        int stt = hs[p].active || hs[p].status == 2 ? MG_NOT_CONVERGED : hs[p].status;
        if (iters) iters[p] = hs[p].iters;
        if (relres) relres[p] = hs[p].relres;
        if (status) status[p] = stt;
        if (stt == MG_ERR_DIVERGED) agg = MG_ERR_DIVERGED;
        else if (stt == MG_NOT_CONVERGED && agg == MG_OK) agg = MG_NOT_CONVERGED;
    }
    MG_TRY(c.join.leave());
    return agg;
}

mg_status mg_last_fallbacks(mg_ctx ctx, int32_t *flags)
{
    clear_error();
    MG_TRY(check_ctx(ctx));
    if (!flags) return set_error(MG_ERR_ARG, "flags is null");
    for (int p = 0; p < ctx->nprob; ++p) flags[p] = p < (int)ctx->fell_back.size() ? ctx->fell_back[p] : 0;
    return MG_OK;
}

mg_status mg_last_solve_ms(mg_ctx ctx, double *ms)
{
    clear_error();
    MG_TRY(check_ctx(ctx));
    if (!ms) return set_error(MG_ERR_ARG, "ms is null");
    *ms = ctx->last_ms;
    return MG_OK;
}

mg_status mg_restencil(mg_ctx ctx, const mg_problem *probs)
{
    clear_error();
    MG_TRY(check_ctx(ctx));
    if (!probs) return set_error(MG_ERR_ARG, "probs is null");
    for (int p = 0; p < ctx->nprob; ++p) {
        if (probs[p].n != ctx->probs[p].n)
            return set_error(MG_ERR_SHAPE, "problem %d: n = %d differs from set-up (%d)", p, probs[p].n, ctx->probs[p].n);
        if (!probs[p].stencil) return set_error(MG_ERR_ARG, "problem %d: stencil is null", p);
    }
    MG_TRY(ctx->join.enter());
    hipStream_t st = ctx->join.internal;
    MG_HIP(hipMemsetAsync(ctx->d_flag, 0, sizeof(int), st));
    for (int p = 0; p < ctx->nprob; ++p) rebuild_problem(*ctx, p, probs[p].stencil, st);
    MG_HIP(hipGetLastError());
    ctx->smoother_ready = false;
    MG_TRY(read_flag(*ctx, st));
    return ctx->join.leave();
}

const char *mg_kernel_name(int32_t k)
{
    static const char *names[MG_NUM_TIMED_KERNELS] = {
        "outer_residual", "check",    "descend",      "ascend",       "bottom",  "smooth_first",
        "residual_restrict", "prolong", "residual", "smooth_apply", "update_u"};
    return (k >= 0 && k < MG_NUM_TIMED_KERNELS) ? names[k] : "";
}

}  // extern "C"

namespace {

// Launches timed kernel k on the finest level's size class of problem 0.
template <typename T>
void launch_timed(mg_ctx_s &c, int k, const SizeClass &cls, const SizeClass &oc, hipStream_t st)
{
    auto *s = (const CycleSlot<T> *)cls.d_slots;
    auto *o = (const OuterSlot<T> *)oc.d_slots;
    const bool cnn = c.opt.smoother == MG_SMOOTHER_CNN;
    const double w = c.opt.omega;
    const int n = cls.n;
    switch (k) {
    case 0: launch_outer_residual<T>(o, oc.nslots, n, c.d_state, st); break;
    case 1: launch_check<T>(o, oc.nslots, c.d_state, c.d_params, 1, st); break;
    case 2:
        if (c.opt.smoother == MG_SMOOTHER_STACK)
            launch_stack_descend<T>(s, cls.nslots, (n - 1) / 2, c.d_state, st);
        else
            launch_descend<T>(s, cls.nslots, n, cnn, w, c.d_state, st, cls.tile[0]);
        break;
    case 3:
        if (c.opt.smoother == MG_SMOOTHER_STACK)
            launch_stack_ascend<T>(s, cls.nslots, n, c.d_state, st);
        else
            launch_ascend<T>(s, cls.nslots, n, cnn, w, c.d_state, st, cls.tile[1]);
        break;
    case 4:
        if (c.opt.smoother == MG_SMOOTHER_STACK)
            launch_stack_bottom<T>((const BottomSlot<T> *)c.bottom.d_slots, c.nprob, c.bottom_top_n, c.opt.nu_pre,
                                   c.opt.nu_post, c.d_state, nullptr, st);
        else
            launch_bottom<T>((const BottomSlot<T> *)c.bottom.d_slots, c.nprob, c.bottom_top_n, cnn, w,
                             c.opt.nu_pre, c.opt.nu_post, c.d_state, nullptr, st);
        break;
    case 5:
        if (c.opt.smoother == MG_SMOOTHER_STACK)
            launch_stack_cycle<T>(s, cls.nslots, n, kStackFirst, c.d_state, st);
        else
            launch_smooth_first<T>(s, cls.nslots, n, cnn, w, c.d_state, st);
        break;
    case 6: launch_residual_restrict<T>(s, cls.nslots, n, c.d_state, st); break;
    case 7: launch_prolong<T>(s, cls.nslots, n, c.d_state, st); break;
    case 8: launch_residual<T>(s, cls.nslots, n, c.d_state, st); break;
    case 9:
        if (c.opt.smoother == MG_SMOOTHER_STACK)
            launch_stack_cycle<T>(s, cls.nslots, n, kStackPost, c.d_state, st);
        else
            launch_smooth_apply<T>(s, cls.nslots, n, cnn, w, c.d_state, st);
        break;
    default: launch_update_u<T>(o, oc.nslots, n, c.d_state, st); break;
    }
}

}  // namespace

extern "C" mg_status mg_time_kernels(mg_ctx ctx, int32_t reps, double *ms)
{
    clear_error();
    MG_TRY(check_ctx(ctx));
    if (!ms || reps < 1) return set_error(MG_ERR_ARG, "need reps >= 1 and an output array");
    MG_TRY(ctx_check_smoother(*ctx));
    mg_ctx_s &c = *ctx;
    const int n0 = c.probs[0].n;
    const SizeClass *cls = nullptr, *oc = nullptr;
    for (const SizeClass &k : c.classes)
        if (k.n == n0) cls = &k;
    for (const SizeClass &k : c.outer)
        if (k.n == n0) oc = &k;
    if (!cls || !oc) return set_error(MG_ERR_STATE, "problem 0 has no level above the bottom kernel's");
    MG_TRY(c.join.enter());
    hipStream_t st = c.join.internal;
    launch_activate(c.d_state, c.nprob, st);
    for (int k = 0; k < MG_NUM_TIMED_KERNELS; ++k) {
        MG_HIP(hipEventRecord(c.t0, st));
        for (int q = 0; q < reps; ++q) {
            if (c.opt.precision == MG_PREC_FP64)
                launch_timed<double>(c, k, *cls, *oc, st);
            else
                launch_timed<float>(c, k, *cls, *oc, st);
        }
        MG_HIP(hipEventRecord(c.t1, st));
        MG_HIP(hipEventSynchronize(c.t1));
        float t = 0.0f;
        MG_HIP(hipEventElapsedTime(&t, c.t0, c.t1));
        ms[k] = (double)t / reps;
    }
    MG_HIP(hipGetLastError());
    return c.join.leave();
}

// ---------------------------------------------------------------- autotuning
namespace mg {
namespace {

static_assert(MG_NUM_TILES == kNumTiles, "tile count of the ABI and of the kernels");

std::string tune_key(const mg_ctx_s &c, int kernel, const SizeClass &k)
{
    char b[160];
    std::snprintf(b, sizeof b, "%s n=%d slots=%d precision=%d smoother=%d", kernel ? "ascend" : "descend", k.n,
                  k.nslots, c.opt.precision, c.opt.smoother);
    return b;
}

template <typename T>
void launch_tile(mg_ctx_s &c, int kernel, const SizeClass &k, int tile, hipStream_t st)
{
    auto *s = (const CycleSlot<T> *)k.d_slots;
    const bool cnn = c.opt.smoother == MG_SMOOTHER_CNN;
    if (kernel == 0)
        launch_descend<T>(s, k.nslots, k.n, cnn, c.opt.omega, c.d_state, st, tile);
    else
        launch_ascend<T>(s, k.nslots, k.n, cnn, c.opt.omega, c.d_state, st, tile);
}

// Cache file: one "key = tile" line per (kernel, level size, batch, precision, smoother).
void read_tune_cache(const char *path, std::map<std::string, int> &known)
{
    FILE *fh = std::fopen(path, "r");
    if (!fh) return;
    char line[256];
    while (std::fgets(line, sizeof line, fh)) {
        char *eq = std::strrchr(line, '=');
        if (!eq || eq == line || eq[-1] != ' ') continue;
        const int t = std::atoi(eq + 1);
        if (t < 0 || t >= kNumTiles) continue;
        known[std::string(line, eq - 1)] = t;
    }
    std::fclose(fh);
}

mg_status write_tune_cache(const char *path, const std::map<std::string, int> &known)
{
    FILE *fh = std::fopen(path, "w");
    if (!fh) return set_error(MG_ERR_ARG, "cannot write the tuning cache %s", path);
    for (const auto &kv : known) std::fprintf(fh, "%s = %d\n", kv.first.c_str(), kv.second);
    std::fclose(fh);
    return MG_OK;
}

}  // namespace
}  // namespace mg

extern "C" mg_status mg_autotune(mg_ctx ctx, int32_t reps, const char *cache)
{
    clear_error();
    MG_TRY(check_ctx(ctx));
    if (reps < 1) return set_error(MG_ERR_ARG, "reps must be >= 1");
    mg_ctx_s &c = *ctx;
    if (!c.fused || c.classes.empty() || c.opt.smoother == MG_SMOOTHER_STACK)
        return MG_OK;  // no fused level kernels with tile choices
    std::map<std::string, int> known;
    if (cache) read_tune_cache(cache, known);
    bool timed = false;
    MG_TRY(c.join.enter());
    hipStream_t st = c.join.internal;
    launch_activate(c.d_state, c.nprob, st);
    for (SizeClass &k : c.classes) {
        for (int kernel = 0; kernel < 2; ++kernel) {
            const std::string key = tune_key(c, kernel, k);
            const auto it = known.find(key);
            if (it != known.end()) {
                k.tile[kernel] = it->second;
                continue;
            }
            double best = 0.0;
            for (int t = 0; t < kNumTiles; ++t) {
                auto launch = [&]() {
                    if (c.opt.precision == MG_PREC_FP64)
                        launch_tile<double>(c, kernel, k, t, st);
                    else
                        launch_tile<float>(c, kernel, k, t, st);
                };
                launch();  // warm-up
                MG_HIP(hipEventRecord(c.t0, st));
                for (int q = 0; q < reps; ++q) launch();
                MG_HIP(hipEventRecord(c.t1, st));
                MG_HIP(hipEventSynchronize(c.t1));
                float ms = 0.0f;
                MG_HIP(hipEventElapsedTime(&ms, c.t0, c.t1));
                k.tile_ms[kernel][t] = (double)ms / reps;
                if (t == 0 || k.tile_ms[kernel][t] < best) {
                    best = k.tile_ms[kernel][t];
                    k.tile[kernel] = t;
                }
            }
            known[key] = k.tile[kernel];
            timed = true;
        }
    }
    MG_HIP(hipGetLastError());
    drop_graph(c);
    MG_TRY(c.join.leave());
    if (cache && timed) MG_TRY(write_tune_cache(cache, known));
    return MG_OK;
}

extern "C" mg_status mg_get_tile(mg_ctx ctx, int32_t kernel, int32_t n, int32_t *tile, double *ms)
{
    clear_error();
    MG_TRY(check_ctx(ctx));
    if (kernel != 0 && kernel != 1) return set_error(MG_ERR_ARG, "kernel must be 0 (descent) or 1 (ascent)");
    for (const SizeClass &k : ctx->classes) {
        if (k.n != n) continue;
        if (tile) *tile = k.tile[kernel];
        if (ms)
            for (int t = 0; t < kNumTiles; ++t) ms[t] = k.tile_ms[kernel][t];
        return MG_OK;
    }
    return set_error(MG_ERR_ARG, "no level of size %d runs the fused kernels in this context", n);
}

extern "C" mg_status mg_set_tile(mg_ctx ctx, int32_t kernel, int32_t n, int32_t tile)
{
    clear_error();
    MG_TRY(check_ctx(ctx));
    if (kernel != 0 && kernel != 1) return set_error(MG_ERR_ARG, "kernel must be 0 (descent) or 1 (ascent)");
    if (tile < 0 || tile >= kNumTiles) return set_error(MG_ERR_ARG, "tile must be in [0, %d)", kNumTiles);
    bool found = n == 0;
    for (SizeClass &k : ctx->classes)
        if (n == 0 || k.n == n) {
            k.tile[kernel] = tile;
            found = true;
        }
    if (!found) return set_error(MG_ERR_ARG, "no level of size %d runs the fused kernels in this context", n);
    drop_graph(*ctx);
    return MG_OK;
}

extern "C" const char *mg_tile_name(int32_t kernel, int32_t tile)
{
    return (kernel == 0 || kernel == 1) && tile >= 0 && tile < kNumTiles ? tile_name(kernel, tile) : "unknown";
}

// ---------------------------------------------------------------- inference
namespace mg {

// Runs the network on one level with the direct (VALU) kernels in type T.
template <typename T>
mg_status infer_level_direct(mg_ctx_s &c, const LevelBuf &L, const T *params, const int *ch, T *scratch,
                             hipStream_t st)
{
    const int64_t v = L.plane;
    T *x0 = scratch;
    T *bufA = x0 + 9 * v;
    T *bufB = bufA + 32 * v;
    const T *A = (const T *)(c.opt.precision == MG_PREC_FP64 ? (const void *)L.A64 : (const void *)L.A32);
    launch_cnn_input<T>(L.n, L.P, v, A, x0, st);
    const T *in = x0;
    int64_t off = 0;
    T *outs[4] = {bufA, bufB, bufA, bufB};
    for (int l = 0; l < 4; ++l) {
        const int cin = ch[l], cout = ch[l + 1];
        const T *w = params + off, *b = params + off + (int64_t)cout * cin * 9;
        off += (int64_t)cout * cin * 9 + cout;
        launch_conv3x3_direct<T>(L.n, L.P, v, cin, cout, w, b, in, outs[l], l < 3, st);
        in = outs[l];
    }
    launch_cnn_output<T>(L.n, L.P, v, A, in, c.opt.omega, (typename SmootherStore<T>::type *)L.H, st);
    MG_HIP(hipGetLastError());
    return MG_OK;
}

mg_status net_params64(mg_net net, hipStream_t st);  // net.cpp
mg_status net_pack_mfma(mg_net net, hipStream_t st);  // net.cpp

}  // namespace mg

namespace mg {

// Runs the network on the smoothing levels of size n (every size when n == 0)
// of every problem, on stream st after the network's pending work; count
// receives the number of levels computed.
mg_status ctx_infer(mg_ctx_s &c, mg_net net, int n, hipStream_t st, int *count)
{
    const bool fp64 = c.opt.precision == MG_PREC_FP64;
    // FP64 (direct path) scratch: input (9) + two ping-pong activation buffers (32 each) on the
    // largest level; the fused MFMA path keeps its activations in LDS
    if (fp64) {
        int64_t vmax = 0;
        for (const ProbBuf &pb : c.probs) vmax = std::max<int64_t>(vmax, pb.lev[0].plane);
        const size_t need = (size_t)vmax * (9 + 32 + 32) * sizeof(double);
        if (need > c.cnn_scratch_bytes) {
            MG_TRY(c.arena.alloc(&c.cnn_scratch, need));
            c.cnn_scratch_bytes = need;
        }
    }
    MG_HIP(hipEventRecord(net->join.ev, net->join.internal));
    MG_HIP(hipStreamWaitEvent(st, net->join.ev, 0));
    if (fp64)
        MG_TRY(net_params64(net, st));
    else
        MG_TRY(net_pack_mfma(net, st));
    int done = 0;
    for (ProbBuf &pb : c.probs) {
        for (int l = 0; l + 1 < pb.nlev; ++l) {
            const LevelBuf &L = pb.lev[l];
            if (n != 0 && L.n != n) continue;
            if (fp64) MG_TRY(infer_level_direct<double>(c, L, net->params64, net->ch, (double *)c.cnn_scratch, st));
            ++done;
        }
    }
    if (!fp64)
        launch_cnn_fused_levels(c.d_cnn_levels, c.n_cnn_levels, c.cnn_tiles, n, net->packed, CnnNetMap{},
                                c.opt.omega, st);
    MG_HIP(hipGetLastError());
    if (count) *count = done;
    return MG_OK;
}

// Inference with one network per level size (sizes[k] takes nets[k]); every smoothing level size of
// the context must be listed, each once.  Mixed precision: one launch over every level.
mg_status ctx_infer_levels(mg_ctx_s &c, const mg_net *nets, const int32_t *sizes, int count, hipStream_t st)
{
    if (count < 1 || count > kMaxNetSizes)
        return set_error(MG_ERR_ARG, "count must be in [1, %d], got %d", kMaxNetSizes, count);
    for (int k = 0; k < count; ++k) {
        if (!nets[k]) return set_error(MG_ERR_ARG, "nets[%d] is null", k);
        for (int q = 0; q < k; ++q)
            if (sizes[q] == sizes[k]) return set_error(MG_ERR_ARG, "size %d is listed twice", sizes[k]);
    }
    auto net_of = [&](int n) -> int {
        for (int k = 0; k < count; ++k)
            if (sizes[k] == n) return k;
        return -1;
    };
    for (int k = 0; k < count; ++k) {
        bool found = false;
        for (const ProbBuf &pb : c.probs)
            for (int l = 0; l + 1 < pb.nlev; ++l) found = found || pb.lev[l].n == sizes[k];
        if (!found) return set_error(MG_ERR_ARG, "no smoothing level of size %d in this context", sizes[k]);
    }
    for (const ProbBuf &pb : c.probs)
        for (int l = 0; l + 1 < pb.nlev; ++l)
            if (net_of(pb.lev[l].n) < 0) return set_error(MG_ERR_ARG, "level size %d has no network", pb.lev[l].n);
    if (c.opt.precision == MG_PREC_FP64) {  // the direct FP64 path runs level by level anyway
        for (int k = 0; k < count; ++k) MG_TRY(ctx_infer(c, nets[k], sizes[k], st, nullptr));
        return MG_OK;
    }
    CnnNetMap map{};
    map.count = count;
    for (int k = 0; k < count; ++k) {
        mg_net net = nets[k];
        MG_HIP(hipEventRecord(net->join.ev, net->join.internal));
        MG_HIP(hipStreamWaitEvent(st, net->join.ev, 0));
        MG_TRY(net_pack_mfma(net, st));
        map.n[k] = sizes[k];
        map.packed[k] = net->packed;
    }
    launch_cnn_fused_levels(c.d_cnn_levels, c.n_cnn_levels, c.cnn_tiles, 0, nets[0]->packed, map, c.opt.omega, st);
    MG_HIP(hipGetLastError());
    return MG_OK;
}

}  // namespace mg

extern "C" mg_status mg_smoother_infer(mg_ctx ctx, mg_net net)
{
    clear_error();
    MG_TRY(check_ctx(ctx));
    if (ctx->opt.smoother == MG_SMOOTHER_STACK)
        return set_error(MG_ERR_STATE, "the stack smoother is not produced by a network (mg_set_stack)");
    if (!net) return set_error(MG_ERR_ARG, "net is null");
    MG_TRY(ctx->join.enter());
    MG_TRY(ctx_infer(*ctx, net, 0, ctx->join.internal, nullptr));
    ctx->smoother_ready = true;
    return ctx->join.leave();
}

extern "C" mg_status mg_smoother_infer_levels(mg_ctx ctx, const mg_net *nets, const int32_t *sizes, int32_t count)
{
    clear_error();
    MG_TRY(check_ctx(ctx));
    if (ctx->opt.smoother == MG_SMOOTHER_STACK)
        return set_error(MG_ERR_STATE, "the stack smoother is not produced by a network (mg_set_stack)");
    if (!nets || !sizes) return set_error(MG_ERR_ARG, "nets and sizes must not be null");
    MG_TRY(ctx->join.enter());
    MG_TRY(ctx_infer_levels(*ctx, nets, sizes, count, ctx->join.internal));
    ctx->smoother_ready = true;
    return ctx->join.leave();
}

extern "C" mg_status mg_smoother_infer_size(mg_ctx ctx, mg_net net, int32_t n)
{
    clear_error();
    MG_TRY(check_ctx(ctx));
    if (ctx->opt.smoother == MG_SMOOTHER_STACK)
        return set_error(MG_ERR_STATE, "the stack smoother is not produced by a network (mg_set_stack)");
    if (!net) return set_error(MG_ERR_ARG, "net is null");
    bool found = false;
    for (const ProbBuf &pb : ctx->probs)
        for (int l = 0; l + 1 < pb.nlev; ++l) found = found || pb.lev[l].n == n;
    if (!found) return set_error(MG_ERR_ARG, "no smoothing level of size %d in this context", n);
    MG_TRY(ctx->join.enter());
    MG_TRY(ctx_infer(*ctx, net, n, ctx->join.internal, nullptr));
    ctx->smoother_ready = true;
    return ctx->join.leave();
}
