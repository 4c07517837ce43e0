"""GPU adaptive training step (Algorithm 2, mg_alpha_step) against the FP64
oracle (oracle/alpha.py), through the C ABI: the loss and dL/dW in FP64, the
parameter gradient of the FP32 network backward, the Adam update, and the
transposed smoother field."""
import numpy as np
import pytest

import mg_inputs
import oracle as ora
from oracle import alpha

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


def _stage(mg, n, specs, seed, lower="random", coarsest=3):
    """A training stage on size n: stencils, fixed smoothers of the levels below
    (random fields near damped Jacobi, or damped Jacobi itself), data, and the
    three contexts of mg_alpha_step."""
    rng = np.random.default_rng(seed)
    As = [ora.stencil_q1_rotated(n, t, e) for t, e in specs]
    B = len(As)
    opt = mg.Options(precision=mg.PREC_FP64, coarsest_n=coarsest,
                     smoother=mg.SMOOTHER_CNN if lower == "random" else mg.SMOOTHER_JACOBI)
    top = mg.Context([_dev(A) for A in As], mg.Options(precision=mg.PREC_FP64, coarsest_n=coarsest))
    A1 = [top.stencil(b, 1) for b in range(B)]
    coarse = mg.Context(A1, opt)
    coarse_t = mg.Context(A1, opt) if lower == "random" else coarse
    lower_fields = [[] for _ in range(B)]
    for b in range(B):
        h = ora.Hierarchy(As[b], coarsest)
        for l in range(1, h.num_levels - 1):
            m = h.level_n(l)
            if lower == "random":
                W = rng.normal(0.0, 0.03, (25, m, m))
                W[12] += 2.0 / 3.0
            else:
                W = np.zeros((25, m, m))
                W[12] = 2.0 / 3.0
            lower_fields[b].append(W)
            if lower == "random":
                Al = coarse.stencil(b, l - 1)
                coarse.set_smoother(b, l - 1, _dev(W))
                coarse_t.set_smoother(b, l - 1, mg.smoother_transpose(Al, _dev(W)))
    f = [mg_inputs.random_field((n, n), seed + 10 + b) for b in range(B)]
    u0 = [rng.normal(size=(n, n)) for _ in range(B)]
    us = [mg_inputs.random_field((n, n), seed + 20 + b) for b in range(B)]
    return As, lower_fields, f, u0, us, top, coarse, coarse_t


def _oracle_dW(As, params, lower_fields, f, u0, us, ks, coarsest=3):
    B = len(As)
    out = []
    total = 0.0
    for A, lower, fb, u0b, usb, k in zip(As, lower_fields, f, u0, us, ks):
        h, hT = ora.Hierarchy(A, coarsest), ora.Hierarchy(A, coarsest)
        for l, Wl in enumerate(lower, start=1):
            h.set_smoother(l, Wl)
            hT.set_smoother(l, alpha.transpose_field(h.stencil(l), Wl))
        W = ora.cnn_forward(A, params)
        L, dW = alpha.loss_and_grad(A, W, h, hT, fb, u0b, usb, k, scale=1.0 / B)
        total += L
        out.append(dW)
    return total, out


@pytest.mark.parametrize("n,ks,lower", [(15, [1, 3, 2], "random"), (31, [4, 1], "random"),
                                        (15, [2, 2], "jacobi"), (7, [3, 1], "random")])
def test_loss_and_dW_match_oracle_fp64(mg, n, ks, lower):
    specs = [(0.3 + 0.7 * b, 10.0 ** (-b - 1)) for b in range(len(ks))]
    As, lower_fields, f, u0, us, top, coarse, coarse_t = _stage(mg, n, specs, seed=n + len(ks), lower=lower)
    params = mg_inputs.cnn_random(5).astype(np.float32)
    net = mg.Net()
    net.set(params)
    res = mg.alpha_step(top, coarse, coarse_t, net, ks, [_dev(x) for x in f], [_dev(x) for x in u0],
                        [_dev(x) for x in us], mg.TrainOptions(precision=0, apply_update=0), want_dW=True)
    L_ref, dW_ref = _oracle_dW(As, params.astype(np.float64), lower_fields, f, u0, us, ks)
    assert res.loss == pytest.approx(L_ref, rel=1e-11)
    for b in range(len(ks)):
        g = res.dW[b].cpu().numpy()
        assert np.abs(g - dW_ref[b]).max() <= 1e-10 * np.abs(dW_ref[b]).max(), b
    assert np.array_equal(net.get(), params)  # apply_update = 0


def test_parameter_gradient_and_adam_match_oracle(mg):
    n, ks = 15, [2, 1, 3]
    specs = [(0.2, 0.05), (1.1, 0.01), (2.5, 0.3)]
    As, lower_fields, f, u0, us, top, coarse, coarse_t = _stage(mg, n, specs, seed=3)
    params = mg_inputs.cnn_random(6).astype(np.float32)
    L_ref, g_ref = alpha.batch_loss_and_grad(As, params.astype(np.float64), lower_fields, f, u0, us, ks)
    net = mg.Net()
    net.set(params)
    args = (top, coarse, coarse_t, net, ks, [_dev(x) for x in f], [_dev(x) for x in u0], [_dev(x) for x in us])
    res = mg.alpha_step(*args, mg.TrainOptions(precision=0, apply_update=0), want_grad=True)
    assert res.loss == pytest.approx(L_ref, rel=1e-11)
    g = res.grad.astype(np.float64)
    # the network backward runs in FP32 (as the high-frequency training step's parity path)
    assert np.linalg.norm(g - g_ref) <= 1e-4 * np.linalg.norm(g_ref)
    assert np.abs(g - g_ref).max() <= 1e-4 * np.abs(g_ref).max()
    p_ref, _, _ = ora.adam_step(params.astype(np.float64), np.zeros(params.size), np.zeros(params.size), g_ref, 1,
                                lr=1e-3)
    res2 = mg.alpha_step(*args, mg.TrainOptions(precision=0, lr=1e-3))
    assert res2.loss == res.loss  # same parameters, same loss, bit for bit
    p = net.get().astype(np.float64)
    big = np.abs(g_ref) > 1e-3 * np.abs(g_ref).max()
    assert np.abs(p - p_ref)[big].max() <= 1e-6


def test_transposed_field_matches_oracle(mg):
    n = 15
    A = ora.stencil_q1_rotated(n, 1.3, 0.02)
    W = np.random.default_rng(1).normal(size=(25, n, n))
    WT = mg.smoother_transpose(_dev(A), _dev(W)).cpu().numpy()
    ref = alpha.transpose_field(A, W)
    assert np.abs(WT - ref).max() <= 1e-14 * np.abs(ref).max()


def test_training_steps_reduce_the_loss(mg):
    n, B = 15, 8
    specs = [(0.4 * b, 10.0 ** (-2 + 0.25 * b)) for b in range(B)]
    As, _, f, u0, us, top, coarse, coarse_t = _stage(mg, n, specs, seed=9)
    net = mg.Net()  # zero parameters: the smoother starts as damped Jacobi
    fd, u0d, usd = [_dev(x) for x in f], [_dev(x) for x in u0], [_dev(x) for x in us]
    ks = [2] * B
    first = mg.alpha_step(top, coarse, coarse_t, net, ks, fd, u0d, usd, mg.TrainOptions(precision=0, lr=0.0)).loss
    # lr = 0 leaves the parameters (Adam with a zero step) and so the loss unchanged
    assert mg.alpha_step(top, coarse, coarse_t, net, ks, fd, u0d, usd,
                         mg.TrainOptions(precision=0, apply_update=0)).loss == first
    net2 = mg.Net()
    net2.set(mg_inputs.cnn_init(2))
    losses = [mg.alpha_step(top, coarse, coarse_t, net2, ks, fd, u0d, usd, mg.TrainOptions(precision=0, lr=3e-3)).loss
              for _ in range(30)]
    assert losses[-1] < 0.95 * losses[0]  # the oracle's own Adam run: 19.13 -> 17.46


def test_adam_trajectory_follows_oracle(mg):
    n, B, steps = 15, 4, 5
    specs = [(0.5 * b, 10.0 ** (-2 + 0.5 * b)) for b in range(B)]
    As, lower_fields, f, u0, us, top, coarse, coarse_t = _stage(mg, n, specs, seed=12)
    params = mg_inputs.cnn_init(3).astype(np.float32)
    ks = [1, 2, 3, 2]
    net = mg.Net()
    net.set(params)
    fd, u0d, usd = [_dev(x) for x in f], [_dev(x) for x in u0], [_dev(x) for x in us]
    p = params.astype(np.float64)
    m, v = np.zeros_like(p), np.zeros_like(p)
    for t in range(1, steps + 1):
        L_ref, g_ref = alpha.batch_loss_and_grad(As, p, lower_fields, f, u0, us, ks)
        p, m, v = ora.adam_step(p, m, v, g_ref, t, lr=3e-3)
        L = mg.alpha_step(top, coarse, coarse_t, net, ks, fd, u0d, usd, mg.TrainOptions(precision=0, lr=3e-3)).loss
        assert L == pytest.approx(L_ref, rel=1e-3), t


def test_arguments(mg):
    n = 15
    As, _, f, u0, us, top, coarse, coarse_t = _stage(mg, n, [(0.5, 0.1), (1.0, 0.2)], seed=4)
    net = mg.Net()
    fd, u0d, usd = [_dev(x) for x in f], [_dev(x) for x in u0], [_dev(x) for x in us]
    o = mg.TrainOptions(precision=0, apply_update=0)
    for ks in ([0, 1], [1, 65]):
        with pytest.raises(mg.MGError) as e:
            mg.alpha_step(top, coarse, coarse_t, net, ks, fd, u0d, usd, o)
        assert e.value.status == mg.MG_ERR_ARG
    with pytest.raises(mg.MGError):  # BF16 training precision is not offered for this loss
        mg.alpha_step(top, coarse, coarse_t, net, [1, 1], fd, u0d, usd, mg.TrainOptions(precision=1))
    with pytest.raises(mg.MGError) as e:  # coarse hierarchy of the wrong size
        mg.alpha_step(top, top, coarse_t, net, [1, 1], fd, u0d, usd, o)
    assert e.value.status == mg.MG_ERR_SHAPE
    mixed = mg.Context([_dev(A) for A in As], mg.Options(precision=mg.PREC_MIXED, coarsest_n=3))
    with pytest.raises(mg.MGError) as e:
        mg.alpha_step(mixed, coarse, coarse_t, net, [1, 1], fd, u0d, usd, o)
    assert e.value.status == mg.MG_ERR_ARG
    # a valid call still works afterwards
    assert mg.alpha_step(top, coarse, coarse_t, net, [1, 2], fd, u0d, usd, o).loss > 0


def test_committed_per_level_networks_beat_jacobi(mg):
    # the checkpoints of the adaptive training (weights/alpha_n*.bin, one network per level size)
    # on problems they were not trained on: fewer cycles than damped Jacobi, to a true 1e-8
    import math
    import os
    from paper_2102_12071_amd.alpha_train import load_nets
    nets = load_nets(os.path.join(os.path.dirname(mg.__file__), "weights"))
    assert sorted(nets) == [7, 15, 31, 63]
    for n, theta, eps, gain in ((255, math.pi / 3, 1e-3, 3.0), (63, math.pi / 6, 0.01, 3.0), (127, 2.0, 0.1, 1.2)):
        A = mg.stencil_q1_rotated(n, theta, eps)
        f = _dev(mg_inputs.rhs_uniform(n, 1))
        iters = {}
        for name, sm in (("alpha", mg.SMOOTHER_CNN), ("jacobi", mg.SMOOTHER_JACOBI)):
            ctx = mg.Context([A], mg.Options(smoother=sm, coarsest_n=3))
            if sm == mg.SMOOTHER_CNN:
                ctx.infer_levels(nets)
            res = ctx.solve([f], 1e-8, 5000)
            assert res.status[0] == 0, (n, name)
            r = f.cpu().numpy() - ora.matvec(A.cpu().numpy(), res.u[0].cpu().numpy())
            assert np.linalg.norm(r) <= 1.01e-8 * np.linalg.norm(f.cpu().numpy())
            iters[name] = int(res.iters[0])
        assert iters["alpha"] * gain < iters["jacobi"], (n, iters)
