"""GPU parity of red-black coarsening (section 6.1) and its two-layer smoother
against the FP64 oracle (oracle/redblack.py), through the C ABI: Galerkin
levels, V-cycles (Jacobi and H = f2(f1), full and checkerboard last levels,
cycles started on a checkerboard level), solves, and the Algorithm 2 loss,
gradient and Adam step."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import mg_inputs
import oracle as ora
from oracle import redblack as rb

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


def _stencil(kind, n):
    if kind == "q1":
        return ora.stencil_q1_rotated(n, math.pi / 3, 1e-2)
    return ora.stencil_cellavg5(n, mg_inputs.lognormal_coefficient(n, 0.1, 1.0, 7))


def _as_matrix(offs, field):
    """The sparse matrix of a footprint field [K, N, N] (row (i, j) couples to (i + dx, j + dy))."""
    K, N, _ = field.shape
    rows, cols, vals = [], [], []
    j, i = np.mgrid[0:N, 0:N]
    for c in range(K):
        dx, dy = offs[c]
        ii, jj = i + dx, j + dy
        ok = (ii >= 0) & (ii < N) & (jj >= 0) & (jj < N) & (field[c] != 0.0)
        rows.append((j * N + i)[ok])
        cols.append((jj * N + ii)[ok])
        vals.append(field[c][ok])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N * N, N * N))


@pytest.mark.parametrize("kind,n,nlev", [("q1", 15, 5), ("q1", 63, 11), ("cell", 63, 9), ("q1", 255, 15)])
def test_galerkin_levels_match_oracle(mg, kind, n, nlev):
    A = _stencil(kind, n)
    h = mg.RedBlack(_dev(A), nlev)
    ref = rb.RBHierarchy(A, nlev)
    assert [(N, k) for N, k, _ in h.shapes] == ref.shapes
    for l in range(nlev):
        offs, field = h.stencil(l)
        M = _as_matrix(offs, field.cpu().numpy())
        D = (M - ref.A[l]).tocoo()
        scale = abs(ref.A[l]).max()
        # level l is a chain of l Galerkin products, each summed in another order than the oracle's
        # sparse products (and with cancellation: rows sum to about zero), so the FP64 rounding
        # difference may grow by about 1e-13 of the level's largest entry per product
        assert (np.abs(D.data).max() if D.nnz else 0.0) <= 1e-13 * (1 + l) * scale, l
    shapes = [(N, k, K) for N, k, K in h.shapes]
    assert shapes[1][2] == 21 and shapes[2][2] == 25  # the footprints grow past 3 x 3


@pytest.mark.parametrize("n,nlev,smoother,nu", [(15, 5, "jacobi", (1, 1)), (15, 5, "stack", (1, 1)),
                                                (15, 4, "stack", (2, 1)), (31, 6, "stack", (1, 2)),
                                                (7, 2, "jacobi", (1, 1)), (127, 13, "stack", (1, 1))])
def test_vcycle_matches_oracle(mg, n, nlev, smoother, nu):
    A = _stencil("q1", n)
    h = mg.RedBlack(_dev(A), nlev)
    ref = rb.RBHierarchy(A, nlev)
    rng = np.random.default_rng(nlev)
    if smoother == "stack":
        for l in range(nlev - 1):
            N = ref.level_n(l)
            phi = rb.jacobi_stack(ref.diag(l)[N // 2, N // 2]) + 0.03 * rng.normal(size=(2, 3, 3))
            ref.set_smoother(l, phi)
            h.set_smoother(l, phi)
    for level in range(min(2, nlev)):
        N = ref.level_n(level)
        r = rng.uniform(-1, 1, (3, N, N)) * ref.masks[level]
        e = h.vcycle(_dev(r), level, *nu).cpu().numpy()
        for v in range(3):
            want = ref.vcycle(r[v], level, *nu)
            assert np.abs(e[v] - want).max() <= 1e-12 * np.abs(want).max(), (level, v)


@pytest.mark.parametrize("smoother", ["jacobi", "stack"])
def test_solve_matches_oracle(mg, smoother):
    n = 63
    A = _stencil("q1", n)
    nlev = 11
    h = mg.RedBlack(_dev(A), nlev)
    ref = rb.RBHierarchy(A, nlev)
    if smoother == "stack":
        rng = np.random.default_rng(5)
        for l in range(nlev - 1):
            N = ref.level_n(l)
            phi = rb.jacobi_stack(ref.diag(l)[N // 2, N // 2]) + 0.01 * rng.normal(size=(2, 3, 3))
            ref.set_smoother(l, phi)
            h.set_smoother(l, phi)
    fs = np.stack([mg_inputs.rhs_uniform(n, s) for s in range(3)])
    res = h.solve(_dev(fs), 1e-10, 3000, history=True)
    for v in range(3):
        _, k, hist, conv = ref.solve(fs[v], 1e-10, 3000)
        assert conv and res.status[v] == 0
        assert int(res.iters[v]) == k
        assert np.allclose(res.history[v, :k + 1], hist, rtol=1e-9, atol=1e-14)
        r = fs[v] - ora.matvec(A, res.u[v].cpu().numpy())
        assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(fs[v]) * 1.0001


def test_solve_from_a_checkerboard_level(mg):
    n = 63
    A = _stencil("q1", n)
    nlev = 9
    h = mg.RedBlack(_dev(A), nlev)
    ref = rb.RBHierarchy(A, nlev)
    f = mg_inputs.rhs_uniform(n, 4) * ref.masks[1]
    res = h.solve(_dev(f), 1e-11, 2000, history=True, level=1)
    _, k, hist, conv = ref.solve(f, 1e-11, 2000, level=1)
    assert conv and res.status[0] == 0 and int(res.iters[0]) == k
    assert np.allclose(res.history[0, :k + 1], hist, rtol=1e-9, atol=1e-14)


def test_weights_rescaled_to_the_level_operator(mg):
    # a_ref > 0: f1 times a_ref / a_C(middle node): the same cycle as the rescaled weights given as is
    n = 31
    A = _stencil("q1", n)
    h1, h2 = mg.RedBlack(_dev(A), 7), mg.RedBlack(_dev(A), 7)
    ref = rb.RBHierarchy(A, 7)
    rng = np.random.default_rng(3)
    r = rng.uniform(-1, 1, (n, n))
    for l in range(6):
        N = ref.level_n(l)
        a_mid = ref.diag(l)[N // 2, N // 2]
        phi = rb.jacobi_stack(1.0) + 0.02 * rng.normal(size=(2, 3, 3))  # made for a_C = 1
        h1.set_smoother(l, phi, a_ref=1.0)
        scaled = phi.copy()
        scaled[0] /= a_mid
        h2.set_smoother(l, scaled)
    e1, e2 = h1.vcycle(_dev(r)).cpu().numpy(), h2.vcycle(_dev(r)).cpu().numpy()
    assert np.abs(e1 - e2).max() <= 1e-13 * np.abs(e2).max()


def test_solve_at_n1023(mg):
    # the benchmark's problem with red-black coarsening and damped Jacobi, V(1,1) to 1e-8: the
    # oracle's own FP64 residual of the returned solution
    n = 1023
    A = ora.stencil_q1_rotated(n, math.pi / 3, 1e-3)
    h = mg.RedBlack(_dev(A), 15)
    assert h.shapes[-1][:2] == (7, "full")
    f = mg_inputs.rhs_uniform(n, 0)
    res = h.solve(_dev(f), 1e-8, 20000)
    assert res.status[0] == 0
    r = f - ora.matvec(A, res.u[0].cpu().numpy())
    assert np.linalg.norm(r) <= 1.0001e-8 * np.linalg.norm(f)


@pytest.mark.parametrize("level", [0, 1, 2])
def test_alpha_step_matches_oracle(mg, level):
    n = 15
    A = _stencil("q1", n)
    nlev = 5
    h = mg.RedBlack(_dev(A), nlev)
    ref = rb.RBHierarchy(A, nlev)
    rng = np.random.default_rng(20 + level)
    for l in range(level + 1, nlev - 1):  # the levels below carry fixed stacks
        N = ref.level_n(l)
        phi = rb.jacobi_stack(ref.diag(l)[N // 2, N // 2]) + 0.02 * rng.normal(size=(2, 3, 3))
        ref.set_smoother(l, phi)
        h.set_smoother(l, phi)
    N = ref.level_n(level)
    mask = ref.masks[level]
    phi = rb.jacobi_stack(ref.diag(level)[N // 2, N // 2]) + 0.05 * rng.normal(size=(2, 3, 3))
    B = 5
    ks = [1, 3, 2, 3, 1]
    f = rng.uniform(-1, 1, (B, N, N)) * mask
    u0 = rng.normal(size=(B, N, N)) * mask
    us = rng.normal(size=(B, N, N)) * mask
    L_ref, g_ref = ref.batch_loss_and_grad(level, phi, list(f), list(u0), list(us), ks)
    st = mg.RBAdam(phi)
    out = mg.rb_alpha_step(h, level, st, ks, _dev(f), _dev(u0), _dev(us),
                           mg.TrainOptions(precision=0, apply_update=0))
    assert out.loss == pytest.approx(L_ref, rel=1e-12)
    assert np.abs(out.grad - g_ref).max() <= 1e-10 * np.abs(g_ref).max()
    for b in range(B):
        Lb = np.linalg.norm(ref.alpha_forward(level, phi, f[b], u0[b], ks[b]) - us[b])
        assert out.losses[b] == pytest.approx(Lb, rel=1e-12)
    # an Adam step on the device = the oracle's Adam with the oracle's gradient (the ABI carries
    # the hyperparameters as FP32: the oracle takes the same rounded values)
    opts = mg.TrainOptions(lr=1e-3, precision=0, apply_update=1)
    mg.rb_alpha_step(h, level, st, ks, _dev(f), _dev(u0), _dev(us), opts)
    f32 = lambda x: float(np.float32(x))
    p1, _, _ = ora.adam_step(phi.reshape(-1), np.zeros(18), np.zeros(18), g_ref, 1, lr=f32(1e-3),
                             beta1=f32(0.9), beta2=f32(0.999), eps=f32(1e-8))
    assert np.abs(st.phi.cpu().numpy() - p1).max() <= 1e-12 * np.abs(p1).max()


def test_errors(mg):
    A = _stencil("q1", 63)
    with pytest.raises(mg.MGError) as ei:
        mg.RedBlack(_dev(A), 4)  # last level: the checkerboard of 31 x 31 (481 points)
    assert ei.value.status == mg.MG_ERR_ARG
    bad = A.copy()
    bad[3][:, 0] = 1.0  # couples to the boundary
    with pytest.raises(mg.MGError):
        mg.RedBlack(_dev(bad), 9)
    h = mg.RedBlack(_dev(A), 9)
    with pytest.raises(mg.MGError):
        h.set_smoother(8, np.zeros(18))  # the last level has no smoother


def test_committed_redblack_smoothers_beat_jacobi_on_their_problem(mg):
    # the red-black alpha-CNN smoothers trained (Algorithm 2, stable selection) for theta = pi/3,
    # eps = 1e-3 at n = 63, applied without retraining at n = 255: fewer cycles than damped Jacobi
    # V(1,1) with the same coarsening, and the oracle's own residual of the solution
    import os
    from paper_2102_12071_amd.rb_train import install, load_run, levels_for
    path = os.path.join(os.path.dirname(mg.__file__), "weights", "rb_theta1.047_eps0.001.json")
    weights, centres, kinds, _ = load_run(path)
    n = 255
    A = ora.stencil_q1_rotated(n, math.pi / 3, 1e-3)
    f = mg_inputs.rhs_uniform(n, 0)
    h = mg.RedBlack(_dev(A), levels_for(n))
    jac = h.solve(_dev(f), 1e-8, 5000)
    install(h, weights, centres, kinds)
    res = h.solve(_dev(f), 1e-8, 5000)
    assert res.status[0] == 0 and jac.status[0] == 0
    assert int(res.iters[0]) < int(jac.iters[0])
    r = f - ora.matvec(A, res.u[0].cpu().numpy())
    assert np.linalg.norm(r) <= 1.0001e-8 * np.linalg.norm(f)
    # and the cycle with those weights is the oracle's
    ref = rb.RBHierarchy(A, levels_for(n))
    e = h.vcycle(_dev(f)).cpu().numpy()
    deepest = {}
    for l in sorted(weights):
        deepest[kinds[l]] = l
    for l in range(ref.num_levels - 1):
        if l in weights:
            ref.set_smoother(l, weights[l])
        else:
            src = deepest[ref.shapes[l][1]]
            N = ref.level_n(l)
            w = weights[src].copy()
            w[0] *= centres[src] / ref.diag(l)[N // 2, N // 2]
            ref.set_smoother(l, w)
    want = ref.vcycle(f)
    assert np.abs(e - want).max() <= 1e-12 * np.abs(want).max()
