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
