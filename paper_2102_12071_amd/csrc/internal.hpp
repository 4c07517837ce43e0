// Host-side internals shared by the runtime translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <string>
#include <vector>

#include "../../include/mgcnn.h"
#include "common.hpp"
#include "launch.hpp"

namespace mg {

// ------------------------------------------------------------ error state
mg_status set_error(mg_status s, const char *fmt, ...);
void clear_error();

#define MG_HIP(call)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            return ::mg::set_error(e_ == hipErrorOutOfMemory ? MG_ERR_OOM : MG_ERR_DEVICE, "%s: %s (%s:%d)", \
                                   #call, hipGetErrorString(e_), __FILE__, __LINE__);                  \
    } while (0)

#define MG_TRY(expr)                                                                                   \
    do {                                                                                               \
        mg_status s_ = (expr);                                                                         \
        if (s_ < 0) return s_;                                                                         \
    } while (0)

// Checks that a gfx950 device is current (once per process).
mg_status require_device();

// Device allocations owned by a context or network, freed together.  New
// chunks are zeroed on the owner's stream (the library's non-blocking stream,
// which the null stream does not order against) and the call waits for it,
// so no later copy or kernel can race the clearing.
struct Arena {
    std::vector<void *> blocks;
    size_t cap = 0, used = 0;  // the last chunk
    hipStream_t stream = nullptr;
    mg_status alloc(void **p, size_t bytes);
    void release();
};

// Joins the library's internal stream to the caller's stream: work the caller
// queued before the call completes first, and the caller's later work waits
// for the library's.
struct StreamJoin {
    hipStream_t user = nullptr, internal = nullptr;
    hipEvent_t ev = nullptr;
    mg_status init(hipStream_t user_stream);
    mg_status enter();   // internal waits for user
    mg_status leave();   // user waits for internal
    void destroy();
};

struct LevelBuf {
    int n = 0, P = 0;
    int64_t plane = 0;
    double *A64 = nullptr;
    float *A32 = nullptr;
    void *H = nullptr;  // 25 planes: bf16 (mixed) or double (FP64)
    void *r = nullptr, *e = nullptr, *s = nullptr;
    void *phi = nullptr;   // stack smoother: 2 x 54 weights (float or double; before and after the coarse
                           // correction), levels above the coarsest
    bool phi_set = false;  // mg_set_stack has installed them
    int *sym = nullptr;    // device flag: the stencil the cycle reads on this level (FP32 in the mixed
                           // cycle, FP64 otherwise) is symmetric
};

struct ProbBuf {
    int n = 0, nlev = 0;
    LevelBuf lev[kMaxLevels];
    double *u = nullptr, *f = nullptr;  // FP64 on the finest level (pitch P)
    double *Ainv = nullptr;
    double *partial = nullptr;
    int nparts = 0;
    int *sym = nullptr;  // device flag: the finest FP64 stencil is symmetric
};

struct SizeClass {
    int n = 0, nslots = 0;
    void *d_slots = nullptr;  // CycleSlot<T>[nslots] or OuterSlot<T>[nslots]
    std::vector<int> probs;   // the problem of each slot
    bool live = true;         // some problem of the class still iterates (launches skip dead classes)
    // the slots the solver launches: all of them, or (once problems stop) a
    // compacted copy holding the iterating problems only
    std::vector<char> host_slots;  // the slot table as uploaded
    size_t slot_bytes = 0;
    void *d_live = nullptr;        // room for the compacted copy
    void *d_run = nullptr;
    int nrun = 0;
    std::vector<int> run_slots;    // which slots d_run holds, in order
    int tile[2] = {0, 0};     // workgroup shape of the fused descent and ascent
    double tile_ms[2][kNumTiles] = {};  // time per launch of each shape at the last autotuning (0: not timed)
};

}  // namespace mg

namespace mg {
struct TrainDraw;
void train_draw_release(mg_net_s &net);
}  // namespace mg

struct mg_net_s {
    mg::StreamJoin join;
    mg::Arena arena;
    int64_t np = 0;
    int nlayers = 4;
    int ch[5] = {9, 32, 32, 32, 25};
    float *params = nullptr;   // FP32 master weights (device)
    float *m = nullptr, *v = nullptr;
    float *grad = nullptr;     // device gradient of the last step
    double *params64 = nullptr;
    void *packed = nullptr;    // weights re-laid for the MFMA kernels (BF16)
    int64_t step = 0;
    bool packed_valid = false;
    // training scratch, grown on demand
    mg::Arena scratch;
    size_t scratch_bytes = 0;
    void *scratch_base = nullptr;
    std::vector<char> host_desc;  // source of the last asynchronous descriptor upload
    mg::TrainDraw *draw = nullptr;  // the captured step of mg_train_step_draw (train.cpp)
};

namespace mg {
// Services of the solver context used by the Krylov driver (context.cpp).
mg_status ctx_check(mg_ctx c);
mg_status ctx_check_vectors(mg_ctx c, const double *const *f, double *const *u);
// MG_ERR_STATE unless the context's smoother can run: the CNN's fields inferred
// or set, the stack's weights installed on every level above the coarsest.
mg_status ctx_check_smoother(const mg_ctx_s &c);
// The coarse contexts of an Algorithm 2 step (alpha.cpp): FP64, one problem per
// problem of top at its level 1 (same order), as many post- as pre-smoothing
// sweeps, the fixed smoothers installed.  name: the argument's name in messages.
mg_status check_alpha_coarse(const mg_ctx_s &top, const mg_ctx_s &c, const char *name);
// Launches only the slots of the given problems from now on (see update_live).
mg_status ctx_set_live(mg_ctx_s &c, const std::vector<char> &active);
// Enqueues e = V(r) of the live problems: level-0 r in, u += e on the finest level.
void ctx_enqueue_cycle(mg_ctx_s &c, hipStream_t st);
// Network inference on the smoothing levels of size n (0: all) of every problem, on st.
mg_status ctx_infer(mg_ctx_s &c, mg_net net, int n, hipStream_t st, int *count);

// Training services of the network (train.cpp).  net_backward_ext: FP32
// forward and backward with the output gradient dL/dy given per problem
// (dout[b]: device [25][n_b*n_b]), writing dL/dparams to net.grad.
mg_status net_backward_ext(mg_net_s &net, int B, const int *n, const double *const *stencil,
                           const float *const *dout, hipStream_t st);
void net_adam(mg_net_s &net, const mg_train_opts &o, hipStream_t st);
mg_status check_train_opts(const mg_train_opts &o);
}  // namespace mg

struct mg_ctx_s {
    mg::StreamJoin join;
    mg::Arena arena;
    mg_options opt{};
    int nprob = 0;
    std::vector<mg::ProbBuf> probs;
    std::vector<mg::SizeClass> classes;  // levels above the coarsest, n descending
    std::vector<mg::SizeClass> outer;    // finest levels, by n
    mg::SizeClass bottom;                // BottomSlot<T>[nprob] (d_slots), one per problem
    int bottom_top_n = 0;                // largest top level of the bottom kernel
    mg::SolveState *d_state = nullptr;
    mg::SolveParams *d_params = nullptr;
    double *d_scalar = nullptr;          // one device double for set-up reductions read by the host
    int *d_flag = nullptr;
    double *d_history = nullptr;
    size_t history_cap = 0;              // doubles
    bool smoother_ready = false;
    bool fused = false;                  // V(1,1): fused level kernels
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    bool graph_stale = false;            // the live set changed: mg_solve re-captures before its next replay
    hipEvent_t t0 = nullptr, t1 = nullptr;
    double last_ms = 0.0;
    // mg_solve: two pinned copies of the per-problem state, each with the event that follows its copy,
    // so that the next check block can be queued before the host reads the last one
    mg::SolveState *h_state = nullptr;   // [2][nprob], hipHostMalloc
    hipEvent_t ev_state[2] = {nullptr, nullptr};
    // CNN inference scratch (direct path)
    void *cnn_scratch = nullptr;
    size_t cnn_scratch_bytes = 0;
    // one-launch MFMA inference (mixed precision): every smoothing level, largest first
    mg::CnnLevelDesc *d_cnn_levels = nullptr;
    int n_cnn_levels = 0, cnn_tiles = 0;
    // flexible-GMRES workspace: 2 * restart + 3 FP64 vectors of the largest
    // finest grid, partial sums and small coefficient arrays
    std::vector<int> fell_back;          // per problem: the last mg_solve switched it to damped Jacobi
    double *kr_vec = nullptr;
    double *kr_small = nullptr;
    int kr_restart = 0;
    // adaptive-training (Algorithm 2) workspace, grown on demand; al_host
    // stages the small tables uploaded with each step
    void *al_ws = nullptr;
    size_t al_bytes = 0;
    std::vector<char> al_host;
};
