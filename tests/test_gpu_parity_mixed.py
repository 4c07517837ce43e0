"""Mixed-precision parity against the FP64 oracle at the stated tolerances:

* iterates: one mixed V(1,1) cycle of the benchmark problem (n = 1023), and k
  mixed V(2,2) Jacobi iterations of the n = 63 problem, within 1e-5 * k of the
  oracle's FP64 iterates (relative 2-norm), the oracle taking the smoother
  fields the context holds (BF16 values, exact in FP64);
* solves with the committed networks (per-level networks of the adaptive
  training, and the single high-frequency network): the oracle runs the FP64
  solve with the same smoother fields; iteration counts agree and every
  iteration's relative residual lies within a factor of 2 of the oracle's;
* inference: the network output y = W - omega * delta_0 of the BF16 MFMA kernel
  within 1e-2 relative (Frobenius, per level) of the oracle's FP64 network, at
  n = 1023 with the committed weights (levels above 255 on sampled patches the
  oracle computes exactly: four nodes of margin cover the four 3x3 layers).
"""
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


def _weights_dir(mg):
    return os.path.join(os.path.dirname(mg.__file__), "weights")


def _per_level_nets(mg):
    from paper_2102_12071_amd.alpha_train import load_nets
    return load_nets(_weights_dir(mg))


def _hf_net(mg):
    net = mg.Net()
    net.load(os.path.join(_weights_dir(mg), "cnn_hf.bin"))
    return net


def _rel2(a, b):
    return float(np.linalg.norm(np.asarray(a) - b) / np.linalg.norm(b))


def _oracle_with_fields(ctx, A, prob=0):
    """The oracle's FP64 hierarchy of A with the context's smoother fields."""
    h = ora.Hierarchy(A)
    assert h.num_levels == ctx.num_levels(prob)
    for l in range(h.num_levels - 1):
        h.set_smoother(l, ctx.smoother(prob, l).cpu().numpy())
    return h


# ------------------------------------------------------------------ iterates
def test_c2_mixed_cycle_within_contract(mg):
    # the benchmark's configuration: per-level networks, autotuned fused kernels, graph replay
    n = 1023
    A = mg.stencil_q1_rotated(n, math.pi / 3, 1e-3)
    ctx = mg.Context([A], mg.Options(smoother=mg.SMOOTHER_CNN))
    ctx.autotune(3)
    ctx.infer_levels(_per_level_nets(mg))
    f = mg_inputs.rhs_uniform(n, 4)
    u = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    ctx.vcycle([_dev(f)], [u])
    h = _oracle_with_fields(ctx, A.cpu().numpy())
    e = h.vcycle(f, 1, 1)
    got = u.cpu().numpy()
    gap = _rel2(got, e)
    print(f"C2 mixed cycle: relative gap {gap:.3e}")
    assert gap <= 1e-5
    # sampled nodes one by one, tile corners and edges of the fused kernels included
    rng = np.random.default_rng(0)
    nodes = list(zip(rng.integers(0, n, 64), rng.integers(0, n, 64)))
    nodes += [(0, 0), (n - 1, n - 1), (0, n - 1), (n - 1, 0), (63, 64), (127, 128), (511, 512)]
    scale = np.abs(e).max()
    for j, i in nodes:
        assert abs(got[j, i] - e[j, i]) <= 1e-5 * scale, (j, i)


def test_c1_mixed_iterates_within_contract(mg):
    p = mg_inputs.config_c1()
    A = ora.stencil_q1_rotated(p.n, p.theta, p.eps)
    f = mg_inputs.rhs_uniform(p.n, p.rhs_seed)
    ctx = mg.Context([_dev(A)], mg.Options(precision=mg.PREC_MIXED, nu_pre=2, nu_post=2))
    h = ora.Hierarchy(A)
    u = torch.zeros((p.n, p.n), dtype=torch.float64, device="cuda")
    fd = _dev(f)
    ref = np.zeros_like(f)
    for k in range(1, 21):
        ctx.vcycle([fd], [u])
        ref = ref + h.vcycle(f - ora.matvec(A, ref), 2, 2)
        gap = _rel2(u.cpu().numpy(), ref)
        assert gap <= 1e-5 * k, (k, gap)


# -------------------------------------------------------------------- solves
def _history_parity(mg, ctx, A64, f, tol, maxit):
    res = ctx.solve([_dev(f)], tol, maxit, history=True)
    h = _oracle_with_fields(ctx, A64)
    u_ora, k_ora, hist_ora, conv = h.solve(f, tol, maxit, 1, 1)
    k_gpu = int(res.iters[0])
    assert conv and res.status[0] == 0
    print(f"iterations: GPU {k_gpu}, oracle {k_ora}")
    assert abs(k_gpu - k_ora) <= max(1, k_ora // 100)
    m = min(k_gpu, k_ora)
    ratio = res.history[0, :m + 1] / hist_ora[:m + 1]
    assert (ratio > 0.5).all() and (ratio < 2.0).all(), (ratio.min(), ratio.max())
    r = f - ora.matvec(A64, res.u[0].cpu().numpy())
    assert np.linalg.norm(r) <= tol * np.linalg.norm(f) * 1.0001
    return k_gpu, k_ora, ratio


@pytest.mark.parametrize("nets", ["per_level", "hf"])
def test_mixed_cnn_solve_history_n255(mg, nets):
    n = 255
    A = ora.stencil_q1_rotated(n, math.pi / 3, 1e-3)
    f = mg_inputs.rhs_uniform(n, 0)
    ctx = mg.Context([_dev(A)], mg.Options(smoother=mg.SMOOTHER_CNN))
    if nets == "per_level":
        ctx.infer_levels(_per_level_nets(mg))
    else:
        ctx.infer(_hf_net(mg))
    _history_parity(mg, ctx, A, f, 1e-8, 5000)


def test_c2_mixed_cnn_solve_history(mg):
    # the headline solve: n = 1023, theta = pi/3, eps = 1e-3, per-level networks, V(1,1) to 1e-8
    n = 1023
    A = mg.stencil_q1_rotated(n, math.pi / 3, 1e-3)
    f = mg_inputs.rhs_uniform(n, 0)
    ctx = mg.Context([A], mg.Options(smoother=mg.SMOOTHER_CNN))
    ctx.autotune(3)
    ctx.infer_levels(_per_level_nets(mg))
    _history_parity(mg, ctx, A.cpu().numpy(), f, 1e-8, 5000)


# ----------------------------------------------------------------- inference
def _patches(m, size=48):
    """Output windows (j0, i0, size) covering the corners, edges and interior of an m x m level."""
    if m <= 255:
        return [(0, 0, m)]
    s = size
    starts = [0, m // 3, m // 2 - s // 2, m - s]
    return [(j, i, s) for j in starts for i in starts]


def _oracle_y_patch(A, params, j0, i0, s):
    """The oracle's network output on rows j0..j0+s-1, columns i0..i0+s-1 of the level with stencil A:
    computed on the window grown by four nodes (clipped at the domain), which the network's four
    zero-padded 3x3 layers cannot see past; the padding at a clipped side is the domain's own."""
    m = A.shape[1]
    w = s + 8  # square windows (the oracle takes square fields), shifted inside the domain
    assert w <= m
    ja = min(max(0, j0 - 4), m - w)
    ia = min(max(0, i0 - 4), m - w)
    W = ora.cnn_forward(A[:, ja:ja + w, ia:ia + w], params)
    y = W[:, j0 - ja:j0 - ja + s, i0 - ia:i0 - ia + s].copy()
    y[12] -= ora.OMEGA
    return y


@pytest.mark.parametrize("nets", ["hf", "per_level"])
def test_bf16_network_output_n1023(mg, nets):
    n = 1023
    A = mg.stencil_q1_rotated(n, math.pi / 3, 1e-3)
    ctx = mg.Context([A], mg.Options(smoother=mg.SMOOTHER_CNN))
    if nets == "hf":
        net = _hf_net(mg)
        by_size = None
    else:
        by_size = _per_level_nets(mg)
        ctx.infer_levels(by_size)
    if nets == "hf":
        ctx.infer(net)
    h = ora.Hierarchy(A.cpu().numpy())
    sizes = sorted(by_size) if by_size else None
    for l in range(h.num_levels - 1):
        m = h.level_n(l)
        if by_size:  # the network of the nearest trained size (ties: the larger), as infer_levels
            key = min(sizes, key=lambda q: (abs(math.log2(q + 1) - math.log2(m + 1)), -q))
            params = by_size[key].get().astype(np.float64)
        else:
            params = net.get().astype(np.float64)
        As = h.stencil(l)
        W_gpu = ctx.smoother(0, l).cpu().numpy()
        num = den = 0.0
        worst = 0.0
        for j0, i0, s in _patches(m):
            s = min(s, m)
            if s == m:
                y_ora = ora.cnn_forward(As, params)
                y_ora[12] -= ora.OMEGA
            else:
                y_ora = _oracle_y_patch(As, params, j0, i0, s)
            y_gpu = W_gpu[:, j0:j0 + s, i0:i0 + s].copy()
            y_gpu[12] -= ora.OMEGA
            num += float(np.sum((y_gpu - y_ora) ** 2))
            den += float(np.sum(y_ora ** 2))
            pt = np.sqrt(np.sum((y_gpu - y_ora) ** 2, axis=0)) / np.maximum(np.sqrt(np.sum(y_ora ** 2, axis=0)), 1e-30)
            worst = max(worst, float(pt.max()))
        rel = math.sqrt(num / den)
        print(f"level {l} (n = {m}): network output relative error {rel:.3e}, worst point {worst:.3e}")
        assert rel <= 1e-2, (l, rel)
