"""GPU training step: HF loss and gradient parity with the FP64 oracle, Adam,
determinism and checkpoint resume (through the C ABI)."""
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
    return mgcnn


def _batch(seed=0):
    specs = [(15, 0.4, 0.01), (31, 2.0, 0.1), (31, 1.2, 0.001), (63, 0.1, 1.0)]
    stencils = [ora.stencil_q1_rotated(n, t, e) for n, t, e in specs]
    # a Galerkin-coarsened variable-coefficient stencil too
    stencils.append(ora.galerkin(ora.stencil_cellavg5(63, mg_inputs.lognormal_coefficient(63, 0.1, 1.0, seed))))
    J = 4
    vecs = [mg_inputs.hf_pool(a.shape[1], J, seed + q).astype(np.float32).astype(np.float64)
            for q, a in enumerate(stencils)]
    return stencils, vecs


def _dev(stencils, vecs):
    st = [torch.tensor(a, dtype=torch.float64, device="cuda") for a in stencils]
    vs = [torch.tensor(v, dtype=torch.float32, device="cuda") for v in vecs]
    return st, vs


def test_loss_and_gradient_match_oracle_fp32(mg):
    stencils, vecs = _batch()
    params = mg_inputs.cnn_random(3)
    L_ref, g_ref = ora.hf_loss(stencils, vecs, params)
    net = mg.Net()
    net.set(params.astype(np.float32))
    st, vs = _dev(stencils, vecs)
    L, g = net.train_step(st, vs, mg.TrainOptions(precision=0, apply_update=0), want_grad=True)
    assert abs(L - L_ref) <= 1e-5 * L_ref
    g = g.astype(np.float64)
    assert np.linalg.norm(g - g_ref) <= 1e-4 * np.linalg.norm(g_ref)
    assert np.abs(g - g_ref).max() <= 1e-4 * np.abs(g_ref).max()
    # no update was applied
    assert np.array_equal(net.get(), params.astype(np.float32))


def test_adam_step_follows_oracle_gradient(mg):
    stencils, vecs = _batch(1)
    params = mg_inputs.cnn_random(4)
    _, g_ref = ora.hf_loss(stencils, vecs, params)
    p_ref, _, _ = ora.adam_step(params, np.zeros_like(params), np.zeros_like(params), g_ref, 1, lr=1e-3)
    net = mg.Net()
    net.set(params.astype(np.float32))
    st, vs = _dev(stencils, vecs)
    net.train_step(st, vs, mg.TrainOptions(precision=0, lr=1e-3))
    p = net.get().astype(np.float64)
    big = np.abs(g_ref) > 1e-3 * np.abs(g_ref).max()
    assert np.abs(p - p_ref)[big].max() <= 1e-6
    assert np.abs(p - params).max() <= 1.0001e-3


def test_training_is_deterministic_and_resumes_from_checkpoint(mg, tmp_path):
    stencils, vecs = _batch(2)
    st, vs = _dev(stencils, vecs)
    params = mg_inputs.cnn_init(5, zero_last=False).astype(np.float32)
    a = mg.Net()
    a.set(params)
    for _ in range(2):
        a.train_step(st, vs, mg.TrainOptions(precision=0))
    path = os.path.join(str(tmp_path), "ck.bin")
    a.save(path)
    la = [a.train_step(st, vs, mg.TrainOptions(precision=0))[0] for _ in range(2)]
    b = mg.Net()
    b.load(path)
    lb = [b.train_step(st, vs, mg.TrainOptions(precision=0))[0] for _ in range(2)]
    assert la == lb
    assert np.array_equal(a.get(), b.get())


def test_training_reduces_the_loss(mg):
    stencils, vecs = _batch(3)
    st, vs = _dev(stencils, vecs)
    net = mg.Net()
    net.set(mg_inputs.cnn_init(0).astype(np.float32))
    losses = [net.train_step(st, vs, mg.TrainOptions(precision=0, lr=2e-3))[0] for _ in range(40)]
    assert losses[-1] < 0.9 * losses[0]
    # the untrained network is damped Jacobi: its loss is the oracle's Jacobi loss
    L0, _ = ora.hf_loss(stencils, vecs, mg_inputs.cnn_init(0), grad=False)
    assert abs(losses[0] - L0) <= 1e-5 * L0


def _cosine(a, b):
    return float(np.dot(a, b) / (np.linalg.norm(a) * np.linalg.norm(b)))


def test_bf16_mfma_loss_and_gradient_close_to_oracle(mg):
    # BF16 activations and weights, FP32 accumulation: compare with the FP64 oracle by angle and norm
    stencils, vecs = _batch(4)
    params = mg_inputs.cnn_random(7)
    L_ref, g_ref = ora.hf_loss(stencils, vecs, params)
    net = mg.Net()
    net.set(params.astype(np.float32))
    st, vs = _dev(stencils, vecs)
    L, g = net.train_step(st, vs, mg.TrainOptions(precision=1, apply_update=0), want_grad=True)
    g = g.astype(np.float64)
    assert abs(L - L_ref) <= 1e-2 * L_ref
    assert _cosine(g, g_ref) >= 0.999
    assert np.linalg.norm(g - g_ref) <= 2e-2 * np.linalg.norm(g_ref)
    # every layer's block of the gradient, not only the largest one
    off = 0
    for l in range(4):
        cin, cout = mg_inputs.CNN_CHANNELS[l], mg_inputs.CNN_CHANNELS[l + 1]
        k = cout * cin * 9 + cout
        assert _cosine(g[off:off + k], g_ref[off:off + k]) >= 0.995, l
        off += k


def test_bf16_training_step_is_deterministic_and_reduces_the_loss(mg):
    stencils, vecs = _batch(5)
    st, vs = _dev(stencils, vecs)
    p0 = mg_inputs.cnn_init(0).astype(np.float32)
    nets = [mg.Net(), mg.Net()]
    for net in nets:
        net.set(p0)
    losses = [[net.train_step(st, vs, mg.TrainOptions(precision=1, lr=2e-3))[0] for _ in range(40)] for net in nets]
    assert losses[0] == losses[1]
    assert np.array_equal(nets[0].get(), nets[1].get())
    assert losses[0][-1] < 0.9 * losses[0][0]


# ------------------------------------------------------- drawn, graph-replayed steps
def _draws(step, B=10, J=4, pool=24):
    rng = np.random.default_rng([77, step])
    n = [31 if q % 3 else 63 for q in range(B)]  # the same size pattern every step
    theta = rng.uniform(0.0, np.pi, B)
    eps = 10.0 ** rng.uniform(-3.0, 0.0, B)
    index = rng.integers(0, pool, (B, J))
    return n, theta, eps, index


def _pools(pool=24):
    return {m: torch.tensor(mg_inputs.hf_pool(m, pool, 5), dtype=torch.float32, device="cuda") for m in (31, 63)}


def _explicit(mg, n, theta, eps, index, pools):
    st = [mg.stencil_q1_rotated(m, t, e) for m, t, e in zip(n, theta, eps)]
    vs = [pools[m][torch.tensor(ix, dtype=torch.long, device="cuda")].contiguous() for m, ix in zip(n, index)]
    return st, vs


@pytest.mark.parametrize("precision", [0, 1])
def test_drawn_step_equals_the_explicit_step(mg, precision):
    # the library's own stencils and vector gather, inside the captured step, give what the caller's
    # stencils (mg_stencil_q1_rotated) and gathered vectors give to mg_train_step
    pools = _pools()
    params = mg_inputs.cnn_random(11).astype(np.float32)
    a, b = mg.Net(), mg.Net()
    a.set(params)
    b.set(params)
    opts = mg.TrainOptions(precision=precision, apply_update=0)
    for step in range(2):
        n, theta, eps, index = _draws(step)
        La, ga = a.train_step_draw(n, theta, eps, pools, index, opts, want_grad=True)
        st, vs = _explicit(mg, n, theta, eps, index, pools)
        Lb, gb = b.train_step(st, vs, opts, want_grad=True)
        assert La == Lb and np.array_equal(ga, gb), (step, La, Lb)
    if precision == 0:  # and the oracle's FP64 loss and gradient of the drawn batch
        stencils = [ora.stencil_q1_rotated(m, t, e) for m, t, e in zip(n, theta, eps)]
        vecs = [pools[m].cpu().numpy()[ix].astype(np.float64) for m, ix in zip(n, index)]
        L_ref, g_ref = ora.hf_loss(stencils, vecs, params.astype(np.float64))
        assert abs(La - L_ref) <= 1e-5 * L_ref
        assert np.linalg.norm(ga - g_ref) <= 1e-4 * np.linalg.norm(g_ref)


def test_drawn_steps_replay_the_graph_like_eager_steps(mg):
    # several replays with new draws and Adam updates, eager device work and synchronisations
    # between them; every step against the same step taken eagerly
    pools = _pools()
    params = mg_inputs.cnn_random(12).astype(np.float32)
    a, b = mg.Net(), mg.Net()
    a.set(params)
    b.set(params)
    opts = mg.TrainOptions(lr=1e-3, precision=1, apply_update=1)
    junk = torch.zeros(1 << 20, device="cuda")
    for step in range(5):
        n, theta, eps, index = _draws(step)
        La, _ = a.train_step_draw(n, theta, eps, pools, index, opts)
        st, vs = _explicit(mg, n, theta, eps, index, pools)
        Lb, _ = b.train_step(st, vs, opts)
        assert La == pytest.approx(Lb, rel=1e-5), step
        pa, pb = a.get(), b.get()
        assert np.abs(pa - pb).max() <= 1e-6 * np.abs(pb).max(), step
        junk.add_(1.0)
        torch.cuda.synchronize()
    # a batch of another structure rebuilds the captured step
    n, theta, eps, index = _draws(9, B=6)
    La, _ = a.train_step_draw(n, theta, eps, pools, index, mg.TrainOptions(precision=1, apply_update=0))
    st, vs = _explicit(mg, n, theta, eps, index, pools)
    Lb, _ = b.train_step(st, vs, mg.TrainOptions(precision=1, apply_update=0))
    assert La == pytest.approx(Lb, rel=1e-5)


def test_drawn_step_rejects_bad_draws(mg):
    pools = _pools()
    net = mg.Net()
    n, theta, eps, index = _draws(0)
    bad = index.copy()
    bad[0, 0] = 24  # past the pool
    with pytest.raises(mg.MGError):
        net.train_step_draw(n, theta, eps, pools, bad)
    with pytest.raises(mg.MGError):
        net.train_step_draw([33] + list(n[1:]), theta, eps, pools, index)  # no pool of size 33
    e2 = np.array(eps)
    e2[1] = 0.0
    with pytest.raises(mg.MGError):
        net.train_step_draw(n, theta, e2, pools, index)
