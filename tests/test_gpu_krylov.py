"""GPU flexible GMRES preconditioned by the V-cycle (mg_solve_fgmres) against
the oracle's FGMRES (oracle/krylov.py), through the C ABI."""
import math

import numpy as np
import pytest

import mg_inputs
import oracle as ora
from oracle.krylov import fgmres

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


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("restart", [30, 4])
def test_fp64_jacobi_matches_oracle(mg, restart):
    n = 63
    A = ora.stencil_q1_rotated(n, math.pi / 6, 0.01)
    f = mg_inputs.rhs_uniform(n, 0)
    ctx = mg.Context([_dev(A)], mg.Options(precision=mg.PREC_FP64))
    res = ctx.solve_fgmres([_dev(f)], 1e-10, 200, restart=restart, history=True)
    h = ora.Hierarchy(A)
    u_ref, k, hist, conv = fgmres(lambda x: ora.matvec(A, x), lambda r: h.vcycle(r, 1, 1), f, 1e-10, 200, restart)
    assert conv and res.status[0] == 0
    assert res.iters[0] == k
    # the residual estimates of both Arnoldi processes agree to rounding (CGS2 + Givens vs MGS + lstsq)
    assert np.allclose(res.history[0, :k + 1], hist, rtol=1e-6, atol=1e-13)
    assert _rel(res.u[0].cpu().numpy(), u_ref) <= 1e-8
    true = np.linalg.norm(f - ora.matvec(A, res.u[0].cpu().numpy())) / np.linalg.norm(f)
    assert true <= 1e-10 and res.relres[0] == pytest.approx(true, rel=1e-6)


def test_fp64_given_smoother_matches_oracle(mg):
    # explicit 5x5 smoother fields on every level (the learned smoother's form)
    n = 127
    A = ora.stencil_q1_rotated(n, 2.0, 0.01)
    h = ora.Hierarchy(A)
    ctx = mg.Context([_dev(A)], mg.Options(precision=mg.PREC_FP64, smoother=mg.SMOOTHER_CNN))
    rng = np.random.default_rng(7)
    for l in range(h.num_levels - 1):
        m = h.level_n(l)
        W = rng.normal(0.0, 0.03, (25, m, m))
        W[12] += 2.0 / 3.0
        h.set_smoother(l, W)
        ctx.set_smoother(0, l, _dev(W))
    f = mg_inputs.rhs_uniform(n, 3)
    res = ctx.solve_fgmres([_dev(f)], 1e-9, 300, restart=20, history=True)
    u_ref, k, hist, conv = fgmres(lambda x: ora.matvec(A, x), lambda r: h.vcycle(r, 1, 1), f, 1e-9, 300, 20)
    assert conv and res.status[0] == 0 and res.iters[0] == k
    assert np.allclose(res.history[0, :k + 1], hist, rtol=1e-6, atol=1e-13)
    assert _rel(res.u[0].cpu().numpy(), u_ref) <= 1e-7


def test_mixed_cnn_accelerates_the_stationary_cycle(mg):
    # the trained network's smoother in BF16 with the FP32 cycle as the
    # (slightly nonlinear) preconditioner: FGMRES stays correct and needs far
    # fewer cycles than the stationary iteration
    import os
    n = 255
    A = _dev(ora.stencil_q1_rotated(n, math.pi / 3, 1e-3))
    f = mg_inputs.rhs_uniform(n, 0)
    net = mg.Net()
    net.load(os.path.join(os.path.dirname(mg.__file__), "weights", "cnn_hf.bin"))
    out = {}
    for name, sm in (("cnn", mg.SMOOTHER_CNN), ("jacobi", mg.SMOOTHER_JACOBI)):
        ctx = mg.Context([A], mg.Options(smoother=sm))
        if sm == mg.SMOOTHER_CNN:
            ctx.infer(net)
        g = ctx.solve_fgmres([_dev(f)], 1e-8, 500, restart=50)
        s = ctx.solve([_dev(f)], 1e-8, 5000)
        assert g.status[0] == 0 and s.status[0] == 0
        true = np.linalg.norm(f - ora.matvec(ora.stencil_q1_rotated(n, math.pi / 3, 1e-3), g.u[0].cpu().numpy()))
        assert true / np.linalg.norm(f) <= 1e-8
        assert g.iters[0] * 3 < s.iters[0]
        out[name] = int(g.iters[0])
    assert out["cnn"] < out["jacobi"]


def test_batch_equals_single_problem_solves(mg):
    specs = [(63, 0.3, 0.1), (127, 2.0, 0.01), (31, 1.0, 1.0), (7, 0.5, 0.5)]
    As = [_dev(ora.stencil_q1_rotated(n, t, e)) for n, t, e in specs]
    fs = [_dev(mg_inputs.rhs_uniform(n, 30 + q)) for q, (n, _, _) in enumerate(specs)]
    opt = mg.Options(precision=mg.PREC_MIXED)
    res = mg.Context(As, opt).solve_fgmres(fs, 1e-9, 300, restart=10)
    assert (res.status == 0).all()
    for q in range(len(specs)):
        one = mg.Context([As[q]], opt).solve_fgmres([fs[q]], 1e-9, 300, restart=10)
        assert one.iters[0] == res.iters[q]
        assert torch.equal(one.u[0], res.u[q])


def test_arguments_and_zero_rhs(mg):
    n = 15
    A = _dev(ora.stencil_q1_rotated(n, 0.2, 0.3))
    ctx = mg.Context([A])
    f = _dev(mg_inputs.rhs_uniform(n, 0))
    for bad in (0, 257):
        with pytest.raises(mg.MGError):
            ctx.solve_fgmres([f], 1e-8, 10, restart=bad)
    res = ctx.solve_fgmres([torch.zeros_like(f)], 1e-8, 10)
    assert res.iters[0] == 0 and res.status[0] == 0 and not res.u[0].any()
    res = ctx.solve_fgmres([f], 1e-8, 3, restart=2)
    assert res.iters[0] == 3 and res.status[0] == mg.MG_NOT_CONVERGED
    # the stationary solver still works on the same context afterwards
    assert ctx.solve([f], 1e-8, 500).status[0] == 0
