"""Pins of the oracle's Algorithm 2 loss and gradient (oracle/alpha.py)."""
import numpy as np
import pytest

import mg_inputs
import oracle as ora
from oracle import alpha


def _setup(n=15, theta=0.8, eps=0.05, seed=0, lower_scale=0.05):
    A = ora.stencil_q1_rotated(n, theta, eps)
    rng = np.random.default_rng(seed)
    h, hT = ora.Hierarchy(A, 3), ora.Hierarchy(A, 3)
    lower = []
    for l in range(1, h.num_levels - 1):
        m = h.level_n(l)
        Wl = rng.normal(0.0, lower_scale, (25, m, m))
        Wl[12] += 2.0 / 3.0
        h.set_smoother(l, Wl)
        hT.set_smoother(l, alpha.transpose_field(h.stencil(l), Wl))
        lower.append(Wl)
    W = rng.normal(0.0, 0.05, (25, n, n))
    W[12] += 2.0 / 3.0
    f = mg_inputs.random_field((n, n), seed + 1)
    u0 = mg_inputs.random_field((n, n), seed + 2)
    us = mg_inputs.random_field((n, n), seed + 3)
    return A, W, h, hT, lower, f, u0, us


def _dense(apply, n):
    M = np.zeros((n * n, n * n))
    for q in range(n * n):
        e = np.zeros(n * n)
        e[q] = 1.0
        M[:, q] = apply(e.reshape(n, n)).ravel()
    return M


def test_forward_is_the_v_cycle_iteration():
    A, W, h, _, _, f, u0, _ = _setup()
    u, _ = alpha.forward(A, W, h, f, u0, 3)
    h.set_smoother(0, W)
    ref = u0.copy()
    for _ in range(3):
        ref = ref + h.vcycle(f - ora.matvec(A, ref), 1, 1)
    assert np.abs(u - ref).max() <= 1e-12 * np.abs(ref).max()


def test_transposed_field_is_the_dense_transpose():
    n = 7
    A = ora.stencil_q1_rotated(n, 2.1, 0.3)
    W = np.random.default_rng(4).normal(size=(25, n, n))
    H = _dense(lambda x: ora.apply_smoother5(A, W, x), n)
    HT = _dense(lambda x: ora.apply_smoother5(A, alpha.transpose_field(A, W), x), n)
    assert np.abs(HT - H.T).max() <= 1e-13 * np.abs(H).max()


def test_transposed_coarse_cycle_is_the_adjoint():
    A, _, h, hT, _, _, _, _ = _setup(n=31, seed=5)
    rng = np.random.default_rng(6)
    x, y = rng.normal(size=(31, 31)), rng.normal(size=(31, 31))
    lhs = np.sum(alpha.coarse_cycle(h, x) * y)
    rhs = np.sum(x * alpha.coarse_cycle(hT, y))
    assert lhs == pytest.approx(rhs, rel=1e-12)


@pytest.mark.parametrize("k", [1, 3])
def test_gradient_matches_central_differences(k):
    A, W, h, hT, _, f, u0, us = _setup(n=7, seed=11)
    L, dW = alpha.loss_and_grad(A, W, h, hT, f, u0, us, k)
    rng = np.random.default_rng(12)
    for _ in range(12):
        c, j, i = rng.integers(25), rng.integers(7), rng.integers(7)
        eps = 1e-6
        Wp, Wm = W.copy(), W.copy()
        Wp[c, j, i] += eps
        Wm[c, j, i] -= eps
        Lp, _ = alpha.loss_and_grad(A, Wp, h, hT, f, u0, us, k)
        Lm, _ = alpha.loss_and_grad(A, Wm, h, hT, f, u0, us, k)
        fd = (Lp - Lm) / (2 * eps)
        assert dW[c, j, i] == pytest.approx(fd, rel=2e-5, abs=1e-9)


def test_parameter_gradient_matches_central_differences():
    n = 15  # levels 15, 7 (fixed smoother), 3 (coarsest)
    A = ora.stencil_q1_rotated(n, 0.5, 0.2)
    h = ora.Hierarchy(A, 3)
    lower = [np.zeros((25, h.level_n(1), h.level_n(1)))]
    lower[0][12] = 2.0 / 3.0
    lower[0][11] = 0.05
    params = mg_inputs.cnn_random(3).astype(np.float64)
    f = mg_inputs.random_field((n, n), 1)
    u0 = mg_inputs.random_field((n, n), 2)
    us = mg_inputs.random_field((n, n), 3)
    L, g = alpha.batch_loss_and_grad([A], params, [lower], [f], [u0], [us], [2])
    rng = np.random.default_rng(0)
    for idx in rng.choice(params.size, 10, replace=False):
        eps = 1e-6
        p1, p2 = params.copy(), params.copy()
        p1[idx] += eps
        p2[idx] -= eps
        Lp, _ = alpha.batch_loss_and_grad([A], p1, [lower], [f], [u0], [us], [2])
        Lm, _ = alpha.batch_loss_and_grad([A], p2, [lower], [f], [u0], [us], [2])
        assert g[idx] == pytest.approx((Lp - Lm) / (2 * eps), rel=1e-4, abs=1e-9)


def test_exact_coarse_solve_two_grid_special_case():
    # n = 7 with coarsest 3: Psi_c is the exact coarse solve, and with W = 0
    # the cycle is the pure coarse-grid correction P A_c^{-1} R
    n = 7
    A = ora.stencil_q1_rotated(n, 0.9, 0.4)
    h = ora.Hierarchy(A, 3)
    assert h.num_levels == 2
    W = np.zeros((25, n, n))
    f = mg_inputs.random_field((n, n), 3)
    u, _ = alpha.forward(A, W, h, f, np.zeros((n, n)), 1)
    Ac = ora.stencil_to_dense(h.stencil(1))
    rc = ora.restrict_fw(f)
    ec = np.linalg.solve(Ac, rc.ravel()).reshape(3, 3)
    ref = ora.prolong_add(ec, np.zeros((n, n)))
    assert np.abs(u - ref).max() <= 1e-13 * np.abs(ref).max()
