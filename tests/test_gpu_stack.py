"""GPU convolution-stack smoother (the constant-coefficient alpha-CNN of
section 5, H = f5(..f1) + f6) through the C ABI against the FP64 oracle
(oracle/stack.py): the LDS-tiled apply, V-cycles and solves in FP64 and mixed
precision, the Algorithm 2 loss, weight gradient and Adam update, and the
error paths."""
import math

import numpy as np
import pytest

import mg_inputs
import oracle as ora
from oracle import stack as st

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mg():
    from paper_2102_12071_amd import mgcnn
    mgcnn.load_library()
    assert torch.cuda.is_available()
    return mgcnn


def _dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def _scaled(seed, A, f32=False):
    w = mg_inputs.stack_random(seed)
    w[4:] /= A[4].flat[0]
    return w.astype(np.float32).astype(np.float64) if f32 else w


@pytest.mark.parametrize("n,count", [(1, 2), (13, 3), (64, 1), (127, 2), (130, 1)])
def test_stack_apply_matches_oracle(mg, n, count):
    # one tile, several tiles, exact and ragged tile edges in both directions
    w = mg_inputs.stack_random(n)
    x = np.stack([mg_inputs.random_field((n, n), 10 * n + c) for c in range(count)])
    y0 = np.stack([mg_inputs.random_field((n, n), 10 * n + c + 5) for c in range(count)])
    ref = np.stack([st.stack_apply(w, xc) for xc in x])
    got = mg.stack_apply(_dev(w), _dev(x)).cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    y = _dev(y0)
    mg.stack_apply(_dev(w), _dev(x), y, accumulate=True)
    assert np.abs(y.cpu().numpy() - (y0 + ref)).max() <= 1e-13 * np.abs(y0 + ref).max()


def _hierarchy_pair(mg, n, precision, seed, coarsest=7, f32=False):
    A = ora.stencil_q1_rotated(n, 1.1, 0.03)
    h = st.StackHierarchy(A, coarsest)
    ctx = mg.Context([_dev(A)], mg.Options(smoother=mg.SMOOTHER_STACK, precision=precision, coarsest_n=coarsest))
    assert ctx.num_levels(0) == h.num_levels
    for l in range(h.num_levels - 1):
        w = _scaled(seed + l, h.stencils[l], f32)
        h.set_stack(l, w)
        ctx.set_stack(0, l, w)
    return A, h, ctx


@pytest.mark.parametrize("n", [31, 63, 127, 255])
def test_fp64_cycle_matches_oracle(mg, n):
    # n = 31: the whole cycle in the one-workgroup kernel (which adds e to u); larger: the fused
    # stack descend / ascend kernels above it (ragged tiles at 127: 64 x 16 fine tiles, 32 x 8 coarse)
    A, h, ctx = _hierarchy_pair(mg, n, mg.PREC_FP64, 3)
    f = mg_inputs.rhs_uniform(n, 1)
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    ctx.vcycle([_dev(f)], [u])
    ref = h.vcycle(f)
    assert np.abs(u.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("coarsest", [1, 3, 7])
def test_fp64_two_sweep_cycle_matches_oracle(mg, coarsest):
    # V(2,2): repeated sweeps in the step kernels (n = 63) and in the one-workgroup kernel (n <= 31)
    n = 63
    A = ora.stencil_q1_rotated(n, 2.0, 0.2)
    h = st.StackHierarchy(A, coarsest)
    ctx = mg.Context([_dev(A)], mg.Options(smoother=mg.SMOOTHER_STACK, precision=mg.PREC_FP64,
                                           coarsest_n=coarsest, nu_pre=2, nu_post=2))
    for l in range(h.num_levels - 1):
        w = _scaled(90 + l, h.stencils[l])
        h.set_stack(l, w, post=st.stack_transpose(w))
        ctx.set_stack(0, l, w, symmetric=True)
    f = mg_inputs.rhs_uniform(n, 8)
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    ctx.vcycle([_dev(f)], [u])
    ref = h.vcycle(f, nu1=2, nu2=2)
    assert np.abs(u.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()


def test_mixed_cycle_matches_oracle(mg):
    # FP32 inner cycle with the FP32 weights the context holds
    n = 255
    A, h, ctx = _hierarchy_pair(mg, n, mg.PREC_MIXED, 5, f32=True)
    f = mg_inputs.rhs_uniform(n, 2)
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    ctx.vcycle([_dev(f)], [u])
    ref = h.vcycle(f)
    assert np.abs(u.cpu().numpy() - ref).max() <= 2e-5 * np.abs(ref).max()


def test_fp64_solve_matches_oracle_iterates(mg):
    # near-Jacobi stacks (every kernel non-zero) converge; FP64 histories agree per iteration
    n = 63
    A, h, ctx = _hierarchy_pair(mg, n, mg.PREC_FP64, 11)
    f = mg_inputs.rhs_uniform(n, 3)
    u_ref, k, hist, conv = h.solve(f, 1e-10, 300)
    assert conv
    res = ctx.solve([_dev(f)], 1e-10, 300, history=True)
    assert res.status[0] == 0 and int(res.iters[0]) == k
    assert np.allclose(res.history[0, :k + 1], hist, rtol=1e-9, atol=1e-15)
    assert np.abs(res.u[0].cpu().numpy() - u_ref).max() <= 1e-10 * np.abs(u_ref).max()
    fg = ctx.solve_fgmres([_dev(f)], 1e-10, 300)
    assert fg.status[0] == 0 and int(fg.iters[0]) <= k


def _stage(mg, n, B, seed, coarsest=3):
    """One training stage of a single problem with B instances: the top context (B copies of
    the stencil), the coarse contexts with fixed stacks (transposed in coarse_t), data."""
    A = ora.stencil_q1_rotated(n, 0.9, 0.03)
    Ac = ora.galerkin(A)
    hc = st.StackHierarchy(Ac, coarsest)
    top = mg.Context([_dev(A)] * B, mg.Options(precision=mg.PREC_FP64, coarsest_n=coarsest))
    if hc.num_levels > 1:
        opt = mg.Options(smoother=mg.SMOOTHER_STACK, precision=mg.PREC_FP64, coarsest_n=coarsest)
        coarse, coarse_t = mg.Context([_dev(Ac)] * B, opt), mg.Context([_dev(Ac)] * B, opt)
        for l in range(hc.num_levels - 1):
            wl = _scaled(seed + 30 + l, hc.stencils[l])
            hc.set_stack(l, wl)
            for b in range(B):
                coarse.set_stack(b, l, wl)
                coarse_t.set_stack(b, l, wl, transpose=True)
    else:  # the level below is the coarsest: Psi_c is its exact solve, its own transpose
        coarse = coarse_t = mg.Context([_dev(Ac)] * B, mg.Options(precision=mg.PREC_FP64, coarsest_n=coarsest))
    rng = np.random.default_rng(seed)
    f = [mg_inputs.random_field((n, n), seed + 10 + b) for b in range(B)]
    u0 = [rng.normal(size=(n, n)) for _ in range(B)]
    us = [mg_inputs.random_field((n, n), seed + 20 + b) for b in range(B)]
    return A, hc, top, coarse, coarse_t, f, u0, us


@pytest.mark.parametrize("n,ks", [(7, [2, 1]), (15, [3, 1, 2]), (31, [2, 4])])
def test_alpha_step_matches_oracle(mg, n, ks):
    B = len(ks)
    A, hc, top, coarse, coarse_t, f, u0, us = _stage(mg, n, B, 7 * n)
    w = _scaled(n, A)
    L_ref, g_ref = st.batch_loss_and_grad(A, w, hc, f, u0, us, ks)
    state = mg.StackAdam(w)
    opts = mg.TrainOptions(precision=0, lr=1e-3)
    D = lambda xs: [_dev(x) for x in xs]
    res = mg.stack_alpha_step(top, coarse, coarse_t, state, ks, D(f), D(u0), D(us), opts)
    assert res.loss == pytest.approx(L_ref, rel=1e-12)
    for b in range(B):
        Lb, _ = st.alpha_loss_and_grad(A, w, hc, f[b], u0[b], us[b], ks[b])
        assert res.losses[b] == pytest.approx(Lb, rel=1e-12)
    assert np.abs(res.grad - g_ref).max() <= 1e-10 * np.abs(g_ref).max()
    # the Adam update of the first step (lr held as float32 by the options struct)
    p1, _, _ = ora.adam_step(w.reshape(-1), np.zeros(54), np.zeros(54), res.grad, 1, lr=float(np.float32(1e-3)))
    assert np.abs(state.phi.cpu().numpy() - p1).max() <= 1e-14 * np.abs(p1).max()
    assert state.t == 1


def test_alpha_steps_reduce_the_loss(mg):
    # Algorithm 2 from the damped-Jacobi initialisation (f1..f4 random, f5 zero) on a fixed batch
    n, ks = 15, [4, 4, 4, 4]
    A, hc, top, coarse, coarse_t, f, u0, us = _stage(mg, n, 4, 99)
    w = mg_inputs.stack_init(1)
    w[4:] /= A[4].flat[0]
    state = mg.StackAdam(w)
    opts = mg.TrainOptions(precision=0, lr=1e-2)
    fd, u0d, usd = [_dev(x) for x in f], [_dev(x) for x in u0], [_dev(x) for x in us]
    first = mg.stack_alpha_step(top, coarse, coarse_t, state, ks, fd, u0d, usd, opts).loss
    for _ in range(30):
        last = mg.stack_alpha_step(top, coarse, coarse_t, state, ks, fd, u0d, usd, opts).loss
    assert last < 0.95 * first  # the FP64 oracle reaches 0.91 on this batch
    # the weights the GPU reached give the oracle the same loss
    L_ref, _ = st.batch_loss_and_grad(A, state.phi.cpu().numpy(), hc, f, u0, us, ks)
    probe = mg.stack_alpha_step(top, coarse, coarse_t, state, ks, fd, u0d, usd,
                                mg.TrainOptions(precision=0, apply_update=0))
    assert probe.loss == pytest.approx(L_ref, rel=1e-12)


def test_error_paths(mg):
    n = 15
    A = _dev(ora.stencil_q1_rotated(n, 0.5, 0.1))
    jac = mg.Context([A], mg.Options(precision=mg.PREC_FP64))
    with pytest.raises(mg.MGError) as e:
        jac.set_stack(0, 0, np.zeros(54))
    assert e.value.status == mg.MG_ERR_STATE
    ctx = mg.Context([A], mg.Options(smoother=mg.SMOOTHER_STACK, precision=mg.PREC_FP64))
    f = _dev(mg_inputs.rhs_uniform(n, 0))
    with pytest.raises(mg.MGError) as e:  # no weights installed yet
        ctx.solve([f], 1e-8, 10)
    assert e.value.status == mg.MG_ERR_STATE
    with pytest.raises(mg.MGError) as e:
        ctx.smoother(0, 0)
    assert e.value.status == mg.MG_ERR_STATE
    with pytest.raises(mg.MGError) as e:
        ctx.set_stack(0, ctx.num_levels(0) - 1, np.zeros(54))  # the coarsest level has no smoother
    assert e.value.status == mg.MG_ERR_ARG
    with pytest.raises(mg.MGError) as e:
        mg.Context([A], mg.Options(smoother=mg.SMOOTHER_STACK, fallback=1))
    assert e.value.status == mg.MG_ERR_ARG
    x = torch.zeros((2, n, n), dtype=torch.float64, device="cuda")
    with pytest.raises(mg.MGError) as e:
        mg.stack_apply(_dev(np.zeros(54)), x, x)
    assert e.value.status == mg.MG_ERR_ARG
    bad = np.zeros(54)
    bad[3] = math.nan
    with pytest.raises(mg.MGError) as e:
        ctx.set_stack(0, 0, bad)
    assert e.value.status == mg.MG_ERR_ARG


def _committed(mg, name):
    import os
    from paper_2102_12071_amd.stack_train import load_stacks
    return load_stacks(os.path.join(os.path.dirname(mg.__file__), "weights", name))


def test_committed_stacks_cycle_matches_oracle(mg):
    # the trained weights as inputs: FP64 cycle of the library against the oracle's, every level
    # taking the stack of the nearest trained size scaled by its centre entry
    stacks = _committed(mg, "stack_theta0_eps0.01.json")
    n = 127
    A = ora.stencil_q1_rotated(n, 0.0, 0.01)
    ctx = mg.Context([_dev(A)], mg.Options(smoother=mg.SMOOTHER_STACK, precision=mg.PREC_FP64))
    ctx.set_stacks(stacks)
    h = st.StackHierarchy(A, 7)
    for l in range(h.num_levels - 1):
        m = h.stencils[l].shape[1]
        best = min(stacks, key=lambda q: abs(math.log2(q + 1) - math.log2(m + 1)))
        w = stacks[best].copy()
        w[4:] /= h.stencils[l][4].mean()
        h.set_stack(l, w)
    f = mg_inputs.rhs_uniform(n, 5)
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    ctx.vcycle([_dev(f)], [u])
    ref = h.vcycle(f)
    assert np.abs(u.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()


def test_committed_stacks_solve_the_problem_they_were_trained_for(mg):
    # theta = 0, eps = 0.01 (the paper's first test set): mixed precision to 1e-8, the true FP64
    # residual by the oracle, at least 5x fewer cycles than damped Jacobi
    stacks = _committed(mg, "stack_theta0_eps0.01.json")
    n = 255
    A = mg.stencil_q1_rotated(n, 0.0, 0.01)
    f = mg_inputs.rhs_uniform(n, 0)
    iters = {}
    for name, sm in (("stack", mg.SMOOTHER_STACK), ("jacobi", mg.SMOOTHER_JACOBI)):
        ctx = mg.Context([A], mg.Options(smoother=sm))
        if sm == mg.SMOOTHER_STACK:
            ctx.set_stacks(stacks)
        res = ctx.solve([_dev(f)], 1e-8, 5000)
        assert res.status[0] == 0
        r = f - ora.matvec(A.cpu().numpy(), res.u[0].cpu().numpy())
        assert np.linalg.norm(r) <= 1.01e-8 * np.linalg.norm(f)
        iters[name] = int(res.iters[0])
    assert 5 * iters["stack"] < iters["jacobi"], iters


def test_symmetric_cycle_matches_oracle(mg):
    # H before and H^T after the coarse correction on every level (mg_set_stack_post)
    n = 127
    A = ora.stencil_q1_rotated(n, 0.4, 0.05)
    h = st.StackHierarchy(A, 7)
    ctx = mg.Context([_dev(A)], mg.Options(smoother=mg.SMOOTHER_STACK, precision=mg.PREC_FP64))
    for l in range(h.num_levels - 1):
        w = _scaled(40 + l, h.stencils[l])
        h.set_stack(l, w, post=st.stack_transpose(w))
        ctx.set_stack(0, l, w, symmetric=True)
    f = mg_inputs.rhs_uniform(n, 6)
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    ctx.vcycle([_dev(f)], [u])
    ref = h.vcycle(f)
    assert np.abs(u.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("n,ks", [(15, [2, 3]), (31, [3, 1, 2])])
def test_symmetric_alpha_step_matches_oracle(mg, n, ks):
    B = len(ks)
    A = ora.stencil_q1_rotated(n, 0.9, 0.03)
    Ac = ora.galerkin(A)
    hc = st.StackHierarchy(Ac, 3)
    top = mg.Context([_dev(A)] * B, mg.Options(precision=mg.PREC_FP64, coarsest_n=3))
    coarse = mg.Context([_dev(Ac)] * B, mg.Options(smoother=mg.SMOOTHER_STACK, precision=mg.PREC_FP64,
                                                   coarsest_n=3))
    for l in range(hc.num_levels - 1):
        wl = _scaled(60 + l, hc.stencils[l])
        hc.set_stack(l, wl, post=st.stack_transpose(wl))
        for b in range(B):
            coarse.set_stack(b, l, wl, symmetric=True)
    rng = np.random.default_rng(n)
    f = [mg_inputs.random_field((n, n), 70 + b) for b in range(B)]
    u0 = [rng.normal(size=(n, n)) for _ in range(B)]
    us = [mg_inputs.random_field((n, n), 80 + b) for b in range(B)]
    w = _scaled(n + 1, A)
    L_ref, g_ref = st.batch_loss_and_grad(A, w, hc, f, u0, us, ks, symmetric=True)
    state = mg.StackAdam(w)
    D = lambda xs: [_dev(x) for x in xs]
    res = mg.stack_alpha_step(top, coarse, coarse, state, ks, D(f), D(u0), D(us),
                              mg.TrainOptions(precision=0, apply_update=0), symmetric=True)
    assert res.loss == pytest.approx(L_ref, rel=1e-12)
    assert np.abs(res.grad - g_ref).max() <= 1e-10 * np.abs(g_ref).max()


def test_set_stack_post_needs_the_stack_first(mg):
    A = _dev(ora.stencil_q1_rotated(15, 0.5, 0.1))
    ctx = mg.Context([A], mg.Options(smoother=mg.SMOOTHER_STACK, precision=mg.PREC_FP64))
    w = np.zeros(54)
    import ctypes as C
    rc = mg.load_library().mg_set_stack_post(ctx._h, 0, 0, w.ctypes.data_as(C.POINTER(C.c_double)), 0, 0)
    assert rc == mg.MG_ERR_STATE


@pytest.mark.parametrize("name,theta,eps,factor", [("stack_theta0.785_eps0.01_symmetric.json", math.pi / 4, 0.01, 1),
                                                    ("stack_theta1.047_eps0.001_symmetric.json", math.pi / 3, 1e-3, 5)])
def test_committed_symmetric_stacks_converge_where_the_plain_ones_diverge(mg, name, theta, eps, factor):
    # trained with H^T after the coarse correction: converging at n = 255 with fewer cycles than damped
    # Jacobi (factor times fewer), where the same training with H after it diverges; the true FP64
    # residual by the oracle
    import os
    from paper_2102_12071_amd.stack_train import load_stack_run
    stacks, symmetric = load_stack_run(os.path.join(os.path.dirname(mg.__file__), "weights", name))
    assert symmetric
    n = 255
    A = mg.stencil_q1_rotated(n, theta, eps)
    f = mg_inputs.rhs_uniform(n, 0)
    ctx = mg.Context([A], mg.Options(smoother=mg.SMOOTHER_STACK))
    ctx.set_stacks(stacks, symmetric=True)
    res = ctx.solve([_dev(f)], 1e-8, 5000)
    jac = mg.Context([A], mg.Options(smoother=mg.SMOOTHER_JACOBI)).solve([_dev(f)], 1e-8, 5000)
    assert res.status[0] == 0 and jac.status[0] == 0
    r = f - ora.matvec(A.cpu().numpy(), res.u[0].cpu().numpy())
    assert np.linalg.norm(r) <= 1.01e-8 * np.linalg.norm(f)
    assert factor * int(res.iters[0]) < int(jac.iters[0]), (int(res.iters[0]), int(jac.iters[0]))


def test_uneven_batch_matches_individual_solves(mg):
    # problems of three sizes in one context (size classes of the step kernels, bottom slots of
    # different top sizes): each solves as it does alone, to the same iterate and count
    specs = [(31, 0.3, 0.1), (127, 1.2, 0.05), (63, 2.5, 0.02), (127, 0.0, 0.3)]
    As, fs, stack_sets = [], [], []
    for k, (n, th, ep) in enumerate(specs):
        A = ora.stencil_q1_rotated(n, th, ep)
        h = st.StackHierarchy(A, 7)
        ws = []
        for l in range(h.num_levels - 1):
            w = mg_inputs.stack_random(200 + 10 * k + l, 0.01)
            w[4:] /= h.stencils[l][4].flat[0]
            ws.append(w)
        As.append(A)
        fs.append(mg_inputs.rhs_uniform(n, 20 + k))
        stack_sets.append(ws)
    opt = mg.Options(smoother=mg.SMOOTHER_STACK, precision=mg.PREC_FP64)
    batch = mg.Context([_dev(A) for A in As], opt)
    for p, ws in enumerate(stack_sets):
        for l, w in enumerate(ws):
            batch.set_stack(p, l, w)
    res = batch.solve([_dev(f) for f in fs], 1e-10, 3000)
    for p, (A, f, ws) in enumerate(zip(As, fs, stack_sets)):
        one = mg.Context([_dev(A)], opt)
        for l, w in enumerate(ws):
            one.set_stack(0, l, w)
        r1 = one.solve([_dev(f)], 1e-10, 3000)
        assert res.status[p] == 0 and r1.status[0] == 0
        assert int(res.iters[p]) == int(r1.iters[0])
        assert torch.equal(res.u[p], r1.u[0])


def test_committed_symmetric_stacks_precondition_fgmres(mg):
    # the symmetric stack cycle of the benchmark problem as the preconditioner of FGMRES(30): fewer
    # iterations than with the Jacobi cycle, the true FP64 residual by the oracle
    import os
    from paper_2102_12071_amd.stack_train import load_stack_run
    stacks, symmetric = load_stack_run(os.path.join(os.path.dirname(mg.__file__), "weights",
                                                    "stack_theta1.047_eps0.001_symmetric.json"))
    n = 255
    A = mg.stencil_q1_rotated(n, math.pi / 3, 1e-3)
    f = mg_inputs.rhs_uniform(n, 1)
    ctx = mg.Context([A], mg.Options(smoother=mg.SMOOTHER_STACK))
    ctx.set_stacks(stacks, symmetric=symmetric)
    res = ctx.solve_fgmres([_dev(f)], 1e-8, 1000, restart=30)
    jac = mg.Context([A], mg.Options(smoother=mg.SMOOTHER_JACOBI)).solve_fgmres([_dev(f)], 1e-8, 1000, restart=30)
    assert res.status[0] == 0 and jac.status[0] == 0
    r = f - ora.matvec(A.cpu().numpy(), res.u[0].cpu().numpy())
    assert np.linalg.norm(r) <= 1.01e-8 * np.linalg.norm(f)
    assert int(res.iters[0]) < int(jac.iters[0]), (int(res.iters[0]), int(jac.iters[0]))


def test_mixed_symmetric_cycle_matches_oracle(mg):
    # FP32 inner cycle, H before and H^T after the coarse correction (the transposed weights are a
    # permutation of the FP32 weights the context holds)
    n = 255
    A = ora.stencil_q1_rotated(n, 0.8, 0.02)
    h = st.StackHierarchy(A, 7)
    ctx = mg.Context([_dev(A)], mg.Options(smoother=mg.SMOOTHER_STACK, precision=mg.PREC_MIXED))
    for l in range(h.num_levels - 1):
        w = _scaled(120 + l, h.stencils[l], f32=True)
        h.set_stack(l, w, post=st.stack_transpose(w))
        ctx.set_stack(0, l, w, symmetric=True)
    f = mg_inputs.rhs_uniform(n, 9)
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    ctx.vcycle([_dev(f)], [u])
    ref = h.vcycle(f)
    assert np.abs(u.cpu().numpy() - ref).max() <= 2e-5 * np.abs(ref).max()


def test_normalised_weights_take_each_levels_scale(mg):
    # normalised = 1: the library divides f5 and f6 by the level's mean centre entry; the same cycle
    # as the oracle's with the weights scaled by hand
    n = 63
    A = ora.stencil_q1_rotated(n, 0.7, 0.05)
    h = st.StackHierarchy(A)
    ctx = mg.Context([_dev(A)], mg.Options(smoother=mg.SMOOTHER_STACK, precision=mg.PREC_FP64))
    for l in range(h.num_levels - 1):
        w = mg_inputs.stack_random(40 + l)  # made for a_C = 1
        ctx.set_stack(0, l, w, normalised=True)
        ws = w.reshape(6, 3, 3).copy()
        ws[4:] /= h.stencils[l][4].mean()
        h.set_stack(l, ws)
    f = mg_inputs.rhs_uniform(n, 3)
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    ctx.vcycle([_dev(f)], [u])
    e = h.vcycle(f)
    assert np.abs(u.cpu().numpy() - e).max() <= 1e-13 * np.abs(e).max()
