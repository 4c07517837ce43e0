"""Statistical and structural pins of the seeded input generators."""
import math

import numpy as np
import pytest

import mg_inputs


def test_hf_vectors_live_on_high_frequencies():
    n = 15
    V = mg_inputs.hf_pool(n, 8, 0)
    k = np.arange(1, n + 1)
    S = np.sin(np.pi * np.outer(np.arange(n) + 1, k) / (n + 1)) * math.sqrt(2.0 / (n + 1))  # orthonormal DST
    KX, KY = np.meshgrid(k, k)
    low = np.maximum(KX, KY) <= n / 2
    for v in V:
        assert np.linalg.norm(v) == pytest.approx(1.0, abs=1e-14)
        coef = S.T @ v @ S
        assert np.abs(coef[low]).max() < 1e-13


def test_hf_vectors_are_uniform_on_the_subspace_sphere():
    # Theorem 3 of the paper (section 3.1): E(n ||X z||^2) = ||X||_F^2 for z uniform on the
    # unit sphere; on the HF subspace of dimension n_H: E(n_H ||X z||^2) = ||X Pi_H||_F^2
    n = 7
    rng = np.random.default_rng(0)
    X = rng.standard_normal((n * n, n * n))
    k = np.arange(1, n + 1)
    S = np.sin(np.pi * np.outer(np.arange(n) + 1, k) / (n + 1)) * math.sqrt(2.0 / (n + 1))
    KX, KY = np.meshgrid(k, k)
    hi = (np.maximum(KX, KY) > n / 2).ravel()
    basis = np.kron(S, S)[:, hi]            # columns: orthonormal HF modes (index j*n+i)
    nH = basis.shape[1]
    target = np.linalg.norm(X @ basis, "fro") ** 2
    Z = mg_inputs.hf_vectors(n, 20000, rng).reshape(20000, -1)
    samples = nH * np.sum((Z @ X.T) ** 2, axis=1)
    se = samples.std() / math.sqrt(samples.size)
    assert abs(samples.mean() - target) < 3.5 * se


def test_gaussian_random_field_statistics():
    m = 256
    fields = [mg_inputs.gaussian_random_field(m, 0.1, 1.0, s) for s in range(6)]
    g = np.stack(fields)
    assert abs(g.mean()) < 0.15
    assert abs(g.var() - 1.0) < 0.25
    for lag_cells, expect in ((int(0.05 * m), math.exp(-1 / 8)), (int(0.1 * m), math.exp(-1 / 2))):
        c = np.mean(g[:, :, :-lag_cells] * g[:, :, lag_cells:]) / g.var()
        assert abs(c - expect) < 0.1


def test_cnn_init_layout_and_jacobi_start():
    p = mg_inputs.cnn_init(0)
    assert p.size == 28345
    assert np.all(p[-(25 * 32 * 9 + 25):] == 0)
    assert np.all(p.astype(np.float32).astype(np.float64) == p)
    b = 1 / math.sqrt(9 * 9)
    assert np.abs(p[:32 * 9 * 9]).max() <= b


def test_rhs_and_draws_deterministic():
    assert np.array_equal(mg_inputs.rhs_uniform(7, 3), mg_inputs.rhs_uniform(7, 3))
    ns, th, ep = mg_inputs.training_draws(256, 0)
    assert set(ns.tolist()) <= {31, 63} and th.min() >= 0 and th.max() < math.pi
    assert ep.min() >= 1e-3 and ep.max() <= 1.0
    ns, th, ep, seeds = mg_inputs.c5_draws()
    assert ns.size == 512 and set(ns.tolist()) <= {63, 127, 255, 511, 1023}


def test_random_domain_masks():
    rng = np.random.default_rng(0)
    fracs = []
    for _ in range(40):
        m = mg_inputs.random_domain_mask(63, rng)
        assert m.dtype == np.uint8 and m.shape == (63, 63) and set(np.unique(m)) <= {0, 1}
        fracs.append(m.mean())
    # a disk of radius <= 0.3 removes at most 28 % of the square, a corner rectangle at most 49 %
    assert min(fracs) > 0.45 and max(fracs) < 1.0
    assert mg_inputs.random_domain_mask(63, np.random.default_rng(5)).tolist() == \
        mg_inputs.random_domain_mask(63, np.random.default_rng(5)).tolist()
