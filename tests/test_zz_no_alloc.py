"""mg_solve_fgmres_noalloc: the FGMRES solve with its Krylov workspace in the
library's fixed device array gives, through the C ABI, exactly what
mg_solve_fgmres gives (same kernels, same order), on two calls in a row (the
second smaller, after the first left its vectors in the array), allocates no
device memory, and rejects a workspace beyond the array before any work."""
import math
import os

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


def _case(mg, n, theta, eps, smoother, precision):
    A = _dev(ora.stencil_q1_rotated(n, theta, eps))
    ctx = mg.Context([A], mg.Options(smoother=smoother, precision=precision))
    if smoother == mg.SMOOTHER_CNN:
        net = mg.Net()
        net.load(os.path.join(os.path.dirname(mg.__file__), "weights", "cnn_hf.bin"))
        ctx.infer(net)
    return A, ctx


@pytest.mark.parametrize("first,second", [((255, math.pi / 3, 1e-3, 30, "cnn", "mixed"),
                                           (63, math.pi / 6, 0.01, 10, "jacobi", "fp64"))])
def test_noalloc_fgmres_equals_fgmres_on_two_calls(mg, first, second):
    # the array arrives with the library's code object, which the runtime loads when one of its
    # kernels first runs in the process: one small call first, so that device memory measured
    # around each call below shows only what the call itself allocates
    _, warm = _case(mg, 7, 0.5, 0.5, mg.SMOOTHER_JACOBI, mg.PREC_FP64)
    uw = torch.zeros((7, 7), dtype=torch.float64, device="cuda")
    warm.solve_fgmres([_dev(mg_inputs.rhs_uniform(7, 0))], 1e-8, 20, restart=2, u=[uw], noalloc=True)
    for n, theta, eps, restart, sm, prec in (first, second):
        smoother = mg.SMOOTHER_CNN if sm == "cnn" else mg.SMOOTHER_JACOBI
        precision = mg.PREC_MIXED if prec == "mixed" else mg.PREC_FP64
        f = _dev(mg_inputs.rhs_uniform(n, 3))
        # the allocating entry point first, on its own context: its result is the reference, and
        # the runtime has loaded every code object this solve uses before memory is measured
        _, ctx_ref = _case(mg, n, theta, eps, smoother, precision)
        u_ref = torch.zeros((n, n), dtype=torch.float64, device="cuda")
        r_ref = ctx_ref.solve_fgmres([f], 1e-8, 400, restart=restart, history=True, u=[u_ref])
        A, ctx = _case(mg, n, theta, eps, smoother, precision)
        u_static = torch.full((n, n), 7.0, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        # the first FGMRES call on a fresh context: no workspace allocated (the allocating entry
        # point takes 64 MiB of context memory here)
        r_static = ctx.solve_fgmres([f], 1e-8, 400, restart=restart, history=True, u=[u_static], noalloc=True)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
        u2 = torch.zeros((n, n), dtype=torch.float64, device="cuda")
        r2 = ctx.solve_fgmres([f], 1e-8, 400, restart=restart, history=True, u=[u2], noalloc=True)
        assert torch.equal(u2, u_static) and (r2.iters == r_static.iters).all()
        # identical iterates and histories
        assert r_ref.status[0] == 0 and r_static.status[0] == 0
        assert int(r_static.iters[0]) == int(r_ref.iters[0])
        k = int(r_ref.iters[0])
        assert np.array_equal(r_static.history[0, :k + 1], r_ref.history[0, :k + 1])
        assert r_static.relres[0] == r_ref.relres[0]
        assert torch.equal(u_static, u_ref)
        # and the solution is the oracle's: its FP64 residual
        r = mg_inputs.rhs_uniform(n, 3) - ora.matvec(A.cpu().numpy(), u_static.cpu().numpy())
        assert np.linalg.norm(r) <= 1.0001e-8 * np.linalg.norm(mg_inputs.rhs_uniform(n, 3))


def test_noalloc_fgmres_rejects_a_workspace_beyond_the_array(mg):
    n = 1023
    A, ctx = _case(mg, n, 0.3, 0.1, mg.SMOOTHER_JACOBI, mg.PREC_FP64)
    f = _dev(mg_inputs.rhs_uniform(n, 1))
    u = torch.full((n, n), 5.0, dtype=torch.float64, device="cuda")
    with pytest.raises(mg.MGError) as ei:
        ctx.solve_fgmres([f], 1e-8, 50, restart=30, u=[u], noalloc=True)
    assert ei.value.status == mg.MG_ERR_ARG and "workspace" in str(ei.value)
    assert bool((u == 5.0).all())  # nothing written on an error
    # restart 1 fits at n = 1023: 6 vectors of 1023 * 1024 values
    r = ctx.solve_fgmres([f], 1e-3, 20, restart=1, u=[u], noalloc=True)
    assert int(r.iters[0]) >= 1
