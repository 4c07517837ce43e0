"""Fallback of the learned smoother to damped Jacobi (mg_options.fallback):
a problem whose CNN cycle diverges or stalls is switched, per problem, and
still converges; the others are untouched."""
import math

import numpy as np
import pytest

import mg_inputs
import oracle as ora

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


def _install(ctx, mg, prob, n, scale):
    """W = scale * delta_0 on every smoothing level of one problem (scale 0: no smoothing)."""
    levels = ctx.num_levels(prob)
    m = n
    for l in range(levels - 1):
        W = np.zeros((25, m, m))
        W[12] = scale
        ctx.set_smoother(prob, l, _dev(W))
        m = (m - 1) // 2


def _true_relres(A, f, u):
    return np.linalg.norm(f - ora.matvec(A, u)) / np.linalg.norm(f)


def test_diverging_smoother_falls_back_and_converges(mg):
    n = 63
    A = ora.stencil_q1_rotated(n, math.pi / 6, 0.01)
    f = mg_inputs.rhs_uniform(n, 0)
    tol = 1e-9
    # the oracle's FP64 damped-Jacobi V(1,1) solve from u = 0
    _, k_jac, jac_hist, conv = ora.Hierarchy(A).solve(f, tol, 3000, 1, 1)
    assert conv
    for fb in (0, 1):
        ctx = mg.Context([_dev(A)], mg.Options(precision=mg.PREC_FP64, smoother=mg.SMOOTHER_CNN, fallback=fb,
                                               check_every=4))
        _install(ctx, mg, 0, n, 3.0)  # omega = 3: the cycle amplifies the error
        res = ctx.solve([_dev(f)], tol, 3000, history=True)
        if fb == 0:
            assert res.status[0] == mg.MG_ERR_DIVERGED and ctx.fallbacks()[0] == 0
            continue
        assert res.status[0] == 0 and ctx.fallbacks()[0] == 1
        assert _true_relres(A, f, res.u[0].cpu().numpy()) <= tol
        # u restarted from zero with damped Jacobi: after the few diverging cycles (the check that
        # sees the residual at 100 times its best pauses the problem; its history entry is then
        # overwritten by the restart's) the cycles are exactly the Jacobi solve's
        k_cnn = int(res.iters[0]) - k_jac
        assert 1 <= k_cnn <= 10
        assert res.history[0, k_cnn] == pytest.approx(1.0)
        assert np.allclose(res.history[0, k_cnn:int(res.iters[0]) + 1], jac_hist[:k_jac + 1],
                           rtol=1e-9, atol=1e-14)
        # the learned smoother was overwritten: a CNN solve needs inference again
        with pytest.raises(mg.MGError) as ei:
            ctx.solve([_dev(f)], tol, 10)
        assert ei.value.status == mg.MG_ERR_STATE


def test_stalled_smoother_falls_back_and_continues(mg):
    n = 127
    A = ora.stencil_q1_rotated(n, 1.0, 0.05)
    f = mg_inputs.rhs_uniform(n, 1)
    ctx = mg.Context([_dev(A)], mg.Options(smoother=mg.SMOOTHER_CNN, fallback=1, check_every=8))
    _install(ctx, mg, 0, n, 0.0)  # no smoothing: coarse-grid correction alone stalls
    res = ctx.solve([_dev(f)], 1e-8, 5000, history=True)
    assert res.status[0] == 0 and ctx.fallbacks()[0] == 1
    assert _true_relres(A, f, res.u[0].cpu().numpy()) <= 1e-8
    h = res.history[0, :int(res.iters[0]) + 1]
    assert h[20] > 0.01 * h[0]  # the stalled phase made little progress


def test_only_the_failing_problem_of_a_batch_falls_back(mg):
    import os
    specs = [(127, math.pi / 3, 1e-2), (63, 0.4, 0.1), (255, 2.0, 1e-3)]
    As = [_dev(ora.stencil_q1_rotated(n, t, e)) for n, t, e in specs]
    fs = [_dev(mg_inputs.rhs_uniform(n, 40 + q)) for q, (n, _, _) in enumerate(specs)]
    net = mg.Net()
    net.load(os.path.join(os.path.dirname(mg.__file__), "weights", "cnn_hf.bin"))
    opt = mg.Options(smoother=mg.SMOOTHER_CNN, fallback=1, check_every=4)
    ctx = mg.Context(As, opt)
    ctx.infer(net)
    _install(ctx, mg, 1, 63, 3.0)
    res = ctx.solve(fs, 1e-8, 4000)
    assert (res.status == 0).all()
    assert ctx.fallbacks().tolist() == [0, 1, 0]
    for q in (0, 2):  # the untouched problems iterate exactly as when solved alone
        one = mg.Context([As[q]], opt)
        one.infer(net)
        r1 = one.solve([fs[q]], 1e-8, 4000)
        assert r1.iters[0] == res.iters[q] and torch.equal(r1.u[0], res.u[q])


def test_fallback_close_to_maxit_still_gets_its_cycles(mg):
    # a problem paused for the switch spends the rest of its check block without cycling; the
    # solve must still give it maxit cycles in all (maxit = exactly the cycles this solve needs)
    n = 63
    A = ora.stencil_q1_rotated(n, math.pi / 6, 0.01)
    f = mg_inputs.rhs_uniform(n, 0)
    tol = 1e-9
    opt = mg.Options(precision=mg.PREC_FP64, smoother=mg.SMOOTHER_CNN, fallback=1, check_every=16)
    ctx = mg.Context([_dev(A)], opt)
    _install(ctx, mg, 0, n, 3.0)
    free = ctx.solve([_dev(f)], tol, 3000)
    need = int(free.iters[0])
    assert free.status[0] == 0 and ctx.fallbacks()[0] == 1
    ctx = mg.Context([_dev(A)], opt)
    _install(ctx, mg, 0, n, 3.0)
    res = ctx.solve([_dev(f)], tol, need)
    assert res.status[0] == 0 and int(res.iters[0]) == need
    assert torch.equal(res.u[0], free.u[0])
    ctx = mg.Context([_dev(A)], opt)
    _install(ctx, mg, 0, n, 3.0)
    short = ctx.solve([_dev(f)], tol, need - 1)
    assert short.status[0] == mg.MG_NOT_CONVERGED and int(short.iters[0]) == need - 1
