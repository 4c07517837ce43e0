"""Pins of the oracle's CNN forward, HF loss, gradient and Adam against
independent implementations (torch CPU float64) and closed forms."""
import math

import numpy as np
import pytest

import mg_inputs

torch = pytest.importorskip("torch")

CH = mg_inputs.CNN_CHANNELS


def _torch_forward(A, params, omega=2 / 3, ch=CH):
    """Independent forward with torch.nn.functional.conv2d in float64."""
    F = torch.nn.functional
    x = torch.tensor(A / A[4:5], dtype=torch.float64)[None]
    p = torch.as_tensor(params, dtype=torch.float64)
    off = 0
    L = len(ch) - 1
    for l in range(L):
        cin, cout = ch[l], ch[l + 1]
        w = p[off:off + cout * cin * 9].reshape(cout, cin, 3, 3)
        off += cout * cin * 9
        b = p[off:off + cout]
        off += cout
        x = F.conv2d(x, w, b, padding=1)
        if l < L - 1:
            x = F.relu(x)
    W = x[0].clone()
    W[12] += omega
    return W


def _torch_loss(stencils, vectors, params, omega=2 / 3):
    """Independent loss with autograd: returns (loss, grad)."""
    p = torch.tensor(params, dtype=torch.float64, requires_grad=True)
    F = torch.nn.functional
    total = 0.0
    B, J = len(stencils), vectors[0].shape[0]
    for A, V in zip(stencils, vectors):
        n = A.shape[1]
        x = torch.tensor(A / A[4:5], dtype=torch.float64)[None]
        off = 0
        L = len(CH) - 1
        for l in range(L):
            cin, cout = CH[l], CH[l + 1]
            w = p[off:off + cout * cin * 9].reshape(cout, cin, 3, 3)
            off += cout * cin * 9
            b = p[off:off + cout]
            off += cout
            x = F.conv2d(x, w, b, padding=1)
            if l < L - 1:
                x = F.relu(x)
        W = x[0] + omega * torch.nn.functional.one_hot(torch.tensor(12), 25).to(torch.float64)[:, None, None]
        At = torch.tensor(A)
        aC = At[4]
        for v in V:
            vt = torch.tensor(v)
            vp = F.pad(vt, (1, 1, 1, 1))
            Av = sum(At[3 * (dy + 1) + (dx + 1)] * vp[1 + dy:1 + dy + n, 1 + dx:1 + dx + n]
                     for dy in (-1, 0, 1) for dx in (-1, 0, 1))
            Avp = F.pad(Av, (2, 2, 2, 2))
            y = sum(W[5 * (dy + 2) + (dx + 2)] * Avp[2 + dy:2 + dy + n, 2 + dx:2 + dx + n]
                    for dy in range(-2, 3) for dx in range(-2, 3)) / aC
            total = total + torch.linalg.norm(vt - y)
    loss = total / (B * J)
    loss.backward()
    return float(loss.detach()), p.grad.numpy().copy()


def test_param_count(ora):
    assert ora.cnn_num_params(CH) == 28345 == mg_inputs.cnn_param_count(CH)


@pytest.mark.parametrize("kind", ["q1", "cellavg"])
def test_forward_matches_torch_conv2d(ora, kind):
    n = 15
    if kind == "q1":
        A = ora.stencil_q1_rotated(n, 0.9, 0.02)
    else:
        A = ora.galerkin(ora.stencil_cellavg5(2 * n + 1, mg_inputs.lognormal_coefficient(2 * n + 1, 0.2, 1.0, 3)))
    params = mg_inputs.cnn_random(11)
    W = ora.cnn_forward(A, params)
    Wt = _torch_forward(A, params).numpy()
    assert np.abs(W - Wt).max() <= 1e-13 * max(1.0, np.abs(Wt).max())


def test_zero_last_layer_is_jacobi(ora):
    n = 15
    A = ora.stencil_q1_rotated(n, 1.3, 0.001)
    W = ora.cnn_forward(A, mg_inputs.cnn_init(0))
    expect = np.zeros((25, n, n))
    expect[12] = 2.0 / 3.0
    assert np.array_equal(W, expect)


def test_constant_coefficient_gives_constant_output_inside(ora):
    n = 31
    A = ora.stencil_q1_rotated(n, 2.5, 0.01)
    W = ora.cnn_forward(A, mg_inputs.cnn_random(4))
    inner = W[:, 5:-5, 5:-5]
    assert np.abs(inner - inner[:, :1, :1]).max() < 1e-13


def test_loss_is_one_for_zero_smoother(ora):
    # H = 0: omega = 0 and a zero last layer give ||v|| = 1 for every unit vector
    n = 15
    A = ora.stencil_q1_rotated(n, 0.4, 0.1)
    V = mg_inputs.hf_pool(n, 4, 0)
    L, g = ora.hf_loss([A], [V], mg_inputs.cnn_init(0), omega=0.0)
    assert L == pytest.approx(1.0, abs=1e-14)


def test_loss_single_mode_jacobi_closed_form(ora):
    # isotropic Q1, damped Jacobi: ||(I - omega D^-1 A) v_k|| = |1 - omega lambda_k / a_C|
    n = 15
    A = ora.stencil_q1_rotated(n, 0.0, 1.0)
    x = np.arange(n) + 1
    vs, expect = [], []
    for kx, ky in [(9, 2), (15, 15), (12, 8), (3, 14)]:
        a, b = math.pi * kx / (n + 1), math.pi * ky / (n + 1)
        v = np.outer(np.sin(b * x), np.sin(a * x))
        vs.append(v / np.linalg.norm(v))
        lam = (8 - 2 * math.cos(a) - 2 * math.cos(b) - 4 * math.cos(a) * math.cos(b)) / 3
        expect.append(abs(1 - (2 / 3) * lam / (8 / 3)))
    L, _ = ora.hf_loss([A], [np.array(vs)], mg_inputs.cnn_init(0), grad=False)
    assert L == pytest.approx(np.mean(expect), abs=1e-14)


def test_loss_and_gradient_match_torch_autograd(ora):
    stencils = [ora.stencil_q1_rotated(15, 0.3, 0.05), ora.stencil_q1_rotated(7, 2.0, 0.3),
                ora.galerkin(ora.stencil_cellavg5(15, mg_inputs.lognormal_coefficient(15, 0.2, 1.0, 1)))]
    vectors = [mg_inputs.hf_pool(a.shape[1], 3, 5) for a in stencils]
    params = mg_inputs.cnn_random(8)
    L, g = ora.hf_loss(stencils, vectors, params)
    Lt, gt = _torch_loss(stencils, vectors, params)
    assert L == pytest.approx(Lt, rel=1e-13)
    assert np.abs(g - gt).max() <= 1e-11 * np.abs(gt).max()


def test_gradient_central_differences_15x15(ora):
    # FP64 central differences on a 15 x 15 problem, random parameter subset
    n = 15
    A = ora.stencil_q1_rotated(n, 1.0, 0.01)
    V = mg_inputs.hf_pool(n, 4, 9)
    params = mg_inputs.cnn_random(2)
    _, g = ora.hf_loss([A], [V], params)
    rng = np.random.default_rng(0)
    idx = rng.choice(params.size, 40, replace=False)
    idx = np.concatenate([idx, np.arange(params.size - 250, params.size - 225)])  # last layer too
    h = 1e-6
    checked = 0
    for q in idx:
        pp, pm = params.copy(), params.copy()
        pp[q] += h
        pm[q] -= h
        Lp, _ = ora.hf_loss([A], [V], pp, grad=False)
        Lm, _ = ora.hf_loss([A], [V], pm, grad=False)
        fd = (Lp - Lm) / (2 * h)
        scale = max(abs(fd), abs(g[q]), 1e-3 * np.abs(g).max())
        # a ReLU kink inside [p-h, p+h] makes the difference quotient meaningless: then the
        # one-sided quotients disagree and the point is skipped
        L0, _ = ora.hf_loss([A], [V], params, grad=False)
        if abs((Lp - L0) / h - (L0 - Lm) / h) > 1e-4 * scale:
            continue
        assert abs(fd - g[q]) <= 1e-6 * scale + 1e-10
        checked += 1
    assert checked >= 50


def test_adam_first_step_closed_form(ora):
    rng = np.random.default_rng(1)
    p = rng.standard_normal(100)
    g = rng.standard_normal(100)
    p1, m1, v1 = ora.adam_step(p, np.zeros(100), np.zeros(100), g, 1, lr=1e-3)
    assert np.allclose(p1, p - 1e-3 * np.sign(g), atol=1e-10)


def test_adam_matches_torch(ora):
    rng = np.random.default_rng(2)
    p0 = rng.standard_normal(50)
    pt = torch.tensor(p0, requires_grad=True)
    opt = torch.optim.Adam([pt], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for t in range(1, 6):
        g = rng.standard_normal(50)
        pt.grad = torch.tensor(g)
        opt.step()
        p, m, v = ora.adam_step(p, m, v, g, t)
    assert np.allclose(p, pt.detach().numpy(), rtol=0, atol=1e-14)


def test_network_smoother_on_masked_domain(ora):
    # Dirichlet rows (no off-centre coupling) take damped Jacobi; away from them the output is
    # the unmasked network's, since the network sees only 4 nodes around each point
    n = 31
    A = ora.stencil_q1_rotated(n, 0.7, 0.05)
    mask = mg_inputs.domain_mask(n, "cylinder")
    Am = ora.stencil_mask(A, mask)
    params = mg_inputs.cnn_random(11)
    W = ora.cnn_forward(A, params)
    Wm = ora.cnn_forward(Am, params)
    out = mask == 0
    jac = np.zeros(25)
    jac[12] = ora.OMEGA
    assert np.array_equal(Wm[:, out].T, np.tile(jac, (int(out.sum()), 1)))
    # nodes at distance > 5 (Chebyshev) from every outside node: one for the mask's coupling
    # change, four for the network's receptive field
    far = np.ones((n, n), dtype=bool)
    for j, i in zip(*np.nonzero(out)):
        far[max(j - 5, 0):j + 6, max(i - 5, 0):i + 6] = False
    assert far.sum() > 100
    assert np.array_equal(Wm[:, far], W[:, far])
    # the hole's Galerkin images on the coarser levels: off-centre sums not negative either
    h = ora.Hierarchy(Am, 3)
    S = h.stencil(1)
    Wc = ora.cnn_forward(S, params)
    hole = (S.sum(0) - S[4]) >= 0
    assert hole.sum() > 4 and np.array_equal(Wc[:, hole].T, np.tile(jac, (int(hole.sum()), 1)))
    assert not np.array_equal(Wc[:, ~hole], np.zeros_like(Wc[:, ~hole]))


def test_diffusion_rows_take_the_network(ora):
    # Galerkin coarsening keeps the row sums of interior rows at zero, so their off-centre entries
    # sum to -a_C; the rule can only act on rows next to the Dirichlet boundary.  Rotated Q1
    # stencils never trigger it on any level (off-centre sum at most -18 % of a_C on these draws);
    # strongly varying cell-average coefficients can on a boundary row of a very coarse level
    rng = np.random.default_rng(3)
    for n in (31, 63):
        for _ in range(20):
            h = ora.Hierarchy(ora.stencil_q1_rotated(n, rng.uniform(0, math.pi), 10 ** rng.uniform(-4, 0)), 1)
            for l in range(h.num_levels - 1):
                S = h.stencil(l)
                assert ((S.sum(0) - S[4]) / S[4]).max() < -0.15
    for n in (31, 63):
        for s in range(3):
            for L in (0.05, 0.1, 0.3):
                h = ora.Hierarchy(ora.stencil_cellavg5(n, mg_inputs.lognormal_coefficient(n, L, 1.0, s)), 1)
                for l in range(h.num_levels - 1):
                    S = h.stencil(l)
                    m = S.shape[1]
                    off = (S.sum(0) - S[4]) / S[4]
                    inner = off[1:m - 1, 1:m - 1]
                    assert np.allclose(inner, -1.0, atol=1e-9)  # interior rows sum to zero
