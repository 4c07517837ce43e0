"""Pins of the oracle's operators, transfers, Galerkin coarsening, smoothers,
V-cycle and solver against independent constructions and closed forms."""
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import mg_inputs
from tests.independent import (SparseVCycle, fe_q1_matrix, prolongation_2d, restriction_2d,
                               stencil_field_to_csr)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            key, *vals = line.split()
            out.setdefault(key, []).append([float(v) for v in vals])
    return {k: np.array(v) for k, v in out.items()}


def _rotated_cells(n, theta, eps):
    c, s = math.cos(theta), math.sin(theta)
    one = np.ones((n + 1, n + 1))
    return (c * c + eps * s * s) * one, c * s * (1 - eps) * one, (s * s + eps * c * c) * one


def test_matvec_matches_fe_assembly(ora):
    n = 15
    rng = np.random.default_rng(2)
    k11 = rng.uniform(0.5, 1.5, (n + 1, n + 1))
    k22 = rng.uniform(0.5, 1.5, (n + 1, n + 1))
    k12 = rng.uniform(-0.3, 0.3, (n + 1, n + 1))
    A = ora.stencil_q1_cells(n, k11, k12, k22)
    x = rng.standard_normal((n, n))
    y = ora.matvec(A, x)
    y_ref = (fe_q1_matrix(n, k11, k12, k22) @ x.ravel()).reshape(n, n)
    assert np.abs(y - y_ref).max() <= 1e-14 * np.abs(y_ref).max()


def _operator_matrix(fn, nin, nout):
    M = np.zeros((nout * nout, nin * nin))
    for q in range(nin * nin):
        x = np.zeros(nin * nin)
        x[q] = 1.0
        M[:, q] = fn(x.reshape(nin, nin)).ravel()
    return M


def test_transfer_matrices_match_paper_stencils(ora):
    nc = 7
    n = 2 * nc + 1
    R = _operator_matrix(ora.restrict_fw, n, nc)
    P = _operator_matrix(lambda ec: ora.prolong_add(ec, np.zeros((n, n))), nc, n)
    assert np.array_equal(R, restriction_2d(nc).toarray())
    assert np.array_equal(P, prolongation_2d(nc).toarray())
    assert np.array_equal(R, P.T / 4.0)
    g = _golden("paper_transfer_stencils.txt")
    wR = g["restriction"] * g["restriction_scale"][0, 0]
    wP = g["prolongation"] * g["prolongation_scale"][0, 0]
    # row of R for an interior coarse node, column of P for the same node
    I = J = 3
    row = R[J * nc + I].reshape(n, n)[2 * J:2 * J + 3, 2 * I:2 * I + 3]
    col = P[:, J * nc + I].reshape(n, n)[2 * J:2 * J + 3, 2 * I:2 * I + 3]
    assert np.array_equal(row, wR) and np.array_equal(col, wP)


def test_prolongation_reproduces_linear_functions(ora):
    nc = 15
    n = 2 * nc + 1
    H, h = 1.0 / (nc + 1), 1.0 / (n + 1)
    xc = (np.arange(nc) + 1) * H
    xf = (np.arange(n) + 1) * h
    Xc, Yc = np.meshgrid(xc, xc)
    Xf, Yf = np.meshgrid(xf, xf)
    e = ora.prolong_add(0.3 * Xc - 1.7 * Yc + 0.2, np.zeros((n, n)))
    # away from the boundary (where the zero Dirichlet value enters)
    assert np.allclose(e[2:-2, 2:-2], (0.3 * Xf - 1.7 * Yf + 0.2)[2:-2, 2:-2], atol=1e-14)


@pytest.mark.parametrize("kind", ["q1", "cellavg", "random"])
def test_galerkin_matches_sparse_product(ora, kind):
    n = 15
    rng = np.random.default_rng(4)
    if kind == "q1":
        A = ora.stencil_q1_rotated(n, 1.2, 0.01)
    elif kind == "cellavg":
        A = ora.stencil_cellavg5(n, np.exp(rng.standard_normal((n + 1, n + 1))))
    else:
        k11 = rng.uniform(0.5, 1.5, (n + 1, n + 1))
        k22 = rng.uniform(0.5, 1.5, (n + 1, n + 1))
        k12 = rng.uniform(-0.4, 0.4, (n + 1, n + 1))
        A = ora.stencil_q1_cells(n, k11, k12, k22)
    Ac = ora.galerkin(A)
    nc = (n - 1) // 2
    ref = (restriction_2d(nc) @ stencil_field_to_csr(A) @ prolongation_2d(nc)).toarray()
    got = stencil_field_to_csr(Ac).toarray()
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_galerkin_nested_q1_closed_form(ora):
    # nested bilinear spaces: R A P = (1/4) Q1(K) on the coarse grid, every level
    n, theta, eps = 63, 0.9, 0.003
    A = ora.stencil_q1_rotated(n, theta, eps)
    while n > 7:
        Ac = ora.galerkin(A)
        n = (n - 1) // 2
        assert np.abs(Ac - ora.stencil_q1_rotated(n, theta, eps) / 4.0).max() < 1e-15 * 4 ** 3
        A = ora.stencil_q1_rotated(n, theta, eps)


def test_galerkin_textbook_5pt(ora):
    g = _golden("textbook_galerkin_5pt.txt")
    n = 15
    A = ora.stencil_cellavg5(n, np.ones((n + 1, n + 1)))
    assert np.array_equal(A[:, 7, 7].reshape(3, 3), g["fine"][::-1] * g["fine_scale"][0, 0])
    Ac = ora.galerkin(A)
    got = Ac[:, 3, 3].reshape(3, 3)
    assert np.allclose(got, g["coarse"] * g["coarse_scale"][0, 0], atol=1e-15)


def test_cholesky_solve_matches_numpy(ora):
    A = ora.stencil_q1_rotated(7, 0.5, 0.01)
    M = ora.stencil_to_dense(A)
    assert np.array_equal(M, stencil_field_to_csr(A).toarray())
    L = ora.cholesky(M)
    assert np.allclose(L @ L.T, M, atol=1e-14)
    b = np.random.default_rng(0).standard_normal(49)
    x = ora.cholesky_solve(L, b)
    assert np.allclose(x, np.linalg.solve(M, b), rtol=1e-12, atol=1e-14)
    assert np.abs(M @ x - b).max() < 1e-13
    with pytest.raises(np.linalg.LinAlgError):
        ora.cholesky(-M)


def test_stencil5_with_centre_weight_is_jacobi(ora):
    n = 15
    A = ora.stencil_q1_rotated(n, 0.3, 0.05)
    rng = np.random.default_rng(5)
    r, e = rng.standard_normal((n, n)), rng.standard_normal((n, n))
    W = np.zeros((25, n, n))
    W[12] = 2.0 / 3.0
    assert np.allclose(ora.smooth_stencil5(A, W, r, e), ora.smooth_jacobi(A, r, e), rtol=0, atol=1e-15)


def test_jacobi_matches_relaxation_definition(ora):
    # u_{k+1} = (I - M^{-1} A) u_k + M^{-1} f with M = D / omega (section 2.1)
    n = 15
    A = ora.stencil_q1_rotated(n, 1.0, 0.2)
    M = stencil_field_to_csr(A).toarray()
    rng = np.random.default_rng(6)
    r, e = rng.standard_normal(n * n), rng.standard_normal(n * n)
    D = np.diag(M)
    ref = e - (2 / 3) * (M @ e) / D + (2 / 3) * r / D
    assert np.allclose(ora.smooth_jacobi(A, r.reshape(n, n), e.reshape(n, n)).ravel(), ref, atol=1e-14)


def test_stencil5_matches_dense_gather(ora):
    n = 9
    rng = np.random.default_rng(7)
    A = ora.stencil_q1_rotated(n, 2.2, 0.5)
    W = rng.standard_normal((25, n, n))
    x = rng.standard_normal((n, n))
    H = np.zeros((n * n, n * n))
    for j in range(n):
        for i in range(n):
            for k in range(25):
                dy, dx = k // 5 - 2, k % 5 - 2
                if 0 <= i + dx < n and 0 <= j + dy < n:
                    H[j * n + i, (j + dy) * n + i + dx] = W[k, j, i] / A[4, j, i]
    assert np.allclose(ora.apply_smoother5(A, W, x).ravel(), H @ x.ravel(), atol=1e-13)


@pytest.mark.parametrize("kind,mu", [("q1", 0.5), ("5pt", 2.0 / 3.0)])
def test_jacobi_lfa_smoothing_factor(ora, kind, mu):
    # on Dirichlet sine modes of the isotropic operator, a damped-Jacobi sweep with
    # r = 0 multiplies the mode by 1 - omega*lambda/a_C exactly
    n = 63
    if kind == "q1":
        A = ora.stencil_q1_rotated(n, 0.0, 1.0)
        lam = lambda a, b: (8 - 2 * np.cos(a) - 2 * np.cos(b) - 4 * np.cos(a) * np.cos(b)) / 3
        aC = 8.0 / 3.0
    else:
        A = ora.stencil_cellavg5(n, np.ones((n + 1, n + 1)))
        lam = lambda a, b: 4 - 2 * np.cos(a) - 2 * np.cos(b)
        aC = 4.0
    x = np.arange(n) + 1
    worst = 0.0
    for kx, ky in [(1, 1), (40, 3), (32, 1), (63, 63), (20, 50), (33, 2)]:
        a, b = math.pi * kx / (n + 1), math.pi * ky / (n + 1)
        v = np.outer(np.sin(b * x), np.sin(a * x))
        out = ora.smooth_jacobi(A, np.zeros((n, n)), v)
        g = 1 - (2 / 3) * lam(a, b) / aC
        assert np.allclose(out, g * v, atol=1e-13)
    # smoothing factor: max over the high set max(kx, ky) > n/2
    k = np.arange(1, n + 1)
    KX, KY = np.meshgrid(k, k)
    hi = np.maximum(KX, KY) > n / 2
    G = np.abs(1 - (2 / 3) * lam(math.pi * KX / (n + 1), math.pi * KY / (n + 1)) / aC)
    worst = G[hi].max()
    assert abs(worst - mu) < 2e-3 and worst <= mu + 1e-12


def test_jacobi_convergent_smoother_criterion(ora):
    # section 2.1: M convergent in the energy norm iff M^T + M - A is SPD; for M = D/omega
    A = ora.stencil_q1_rotated(15, 0.7, 0.01)
    M = stencil_field_to_csr(A).toarray()
    Mj = np.diag(np.diag(M)) / (2 / 3)
    assert np.linalg.eigvalsh(Mj.T + Mj - M).min() > 0


@pytest.mark.parametrize("nu1,nu2", [(1, 1), (2, 1), (0, 2)])
def test_two_level_cycle_equals_dense_operator(ora, nu1, nu2):
    n = 15
    A = ora.stencil_q1_rotated(n, 0.8, 0.05)
    mg = ora.Hierarchy(A, coarsest_n=7)
    assert mg.num_levels == 2
    M = stencil_field_to_csr(A).toarray()
    P, R = prolongation_2d(7).toarray(), restriction_2d(7).toarray()
    Ac = R @ M @ P
    S = np.eye(n * n) - (2 / 3) * M / np.diag(M)[:, None]
    E = np.linalg.matrix_power(S, nu2) @ (np.eye(n * n) - P @ np.linalg.solve(Ac, R @ M)) @ np.linalg.matrix_power(S, nu1)
    Ecode = np.zeros_like(E)
    for q in range(n * n):
        x = np.zeros(n * n)
        x[q] = 1.0
        Ecode[:, q] = x - mg.vcycle((M @ x).reshape(n, n), nu1, nu2).ravel()
    assert np.abs(Ecode - E).max() < 1e-13


def test_vcycle_spectral_radius_matches_observed_rate(ora):
    n = 15
    A = ora.stencil_q1_rotated(n, 1.0, 0.01)
    mg = ora.Hierarchy(A, coarsest_n=3)
    M = stencil_field_to_csr(A).toarray()
    E = np.zeros((n * n, n * n))
    for q in range(n * n):
        x = np.zeros(n * n)
        x[q] = 1.0
        E[:, q] = x - mg.vcycle((M @ x).reshape(n, n), 1, 1).ravel()
    rho = np.abs(np.linalg.eigvals(E)).max()
    f = np.random.default_rng(0).uniform(-1, 1, (n, n))
    _, k, hist, conv = mg.solve(f, 1e-300, 80, 1, 1)
    rate = (hist[80] / hist[60]) ** (1 / 20)
    assert abs(rate - rho) < 2e-3


@pytest.mark.parametrize("cfg", ["c1_v22", "c1_v11", "iso_v11", "cellavg"])
def test_solver_matches_sparse_vcycle(ora, cfg):
    # an independent assembled-matrix implementation (scipy) gives the same history
    if cfg == "cellavg":
        n = 31
        a = mg_inputs.lognormal_coefficient(n, 0.1, 1.0, 7)
        A = ora.stencil_cellavg5(n, a)
        nu, tol, maxit = (1, 1), 1e-10, 200
    else:
        n = 63
        theta, eps = (math.pi / 6, 0.01) if cfg.startswith("c1") else (0.0, 1.0)
        A = ora.stencil_q1_rotated(n, theta, eps)
        nu = (2, 2) if cfg.endswith("v22") else (1, 1)
        tol, maxit = 1e-10, 400
    f = mg_inputs.rhs_uniform(n, 0)
    mg = ora.Hierarchy(A, coarsest_n=7)
    u, k, hist, conv = mg.solve(f, tol, maxit, *nu)
    ref = SparseVCycle(stencil_field_to_csr(A), n, 7)
    u_ref, hist_ref = ref.solve(f.ravel(), tol, maxit, *nu)
    assert conv and k == len(hist_ref) - 1
    assert np.allclose(hist, hist_ref, rtol=1e-9, atol=1e-15)
    assert np.abs(u.ravel() - u_ref).max() <= 1e-10 * np.abs(u_ref).max()


def test_c1_iteration_count_and_rate(ora):
    # C1: Jacobi V(2,2) on (pi/6, 0.01), n = 63, to 1e-10
    p = mg_inputs.config_c1()
    A = ora.stencil_q1_rotated(p.n, p.theta, p.eps)
    mg = ora.Hierarchy(A)
    u, k, hist, conv = mg.solve(mg_inputs.rhs_uniform(p.n, p.rhs_seed), 1e-10, 1000, 2, 2)
    assert conv and 120 <= k <= 180
    rate = (hist[k] / hist[k - 20]) ** (1 / 20)
    assert 0.8 < rate < 0.95


def test_isotropic_vcycle_factor(ora):
    n = 63
    mg = ora.Hierarchy(ora.stencil_q1_rotated(n, 0.0, 1.0))
    _, k, hist, conv = mg.solve(mg_inputs.rhs_uniform(n, 0), 1e-10, 100, 2, 2)
    rate = (hist[k] / hist[k - 4]) ** 0.25
    assert conv and rate < 0.15


def test_solution_matches_dense_solve(ora):
    n = 31
    A = ora.stencil_q1_rotated(n, 2.0, 0.05)
    f = mg_inputs.rhs_uniform(n, 1)
    u, k, hist, conv = ora.Hierarchy(A).solve(f, 1e-12, 2000, 1, 1)
    u_ref = np.linalg.solve(stencil_field_to_csr(A).toarray(), f.ravel())
    assert conv
    assert np.linalg.norm(u.ravel() - u_ref) <= 1e-9 * np.linalg.norm(u_ref)


def test_hierarchy_rejects_bad_sizes(ora):
    with pytest.raises(ValueError):
        ora.Hierarchy(ora.stencil_q1_rotated(14, 0.1, 0.1))
    with pytest.raises(ValueError):
        ora.Hierarchy(-ora.stencil_q1_rotated(15, 0.1, 0.1))


def test_jacobi_per_eigenvector_factor(ora):
    # the smoothing-property measure of section 6 (the factor ||v - H A v|| of each unit eigenvector v
    # of A): for damped Jacobi on a constant-diagonal stencil it is |1 - omega lambda / a_C| exactly,
    # from an eigendecomposition made independently of the oracle's smoother routine
    n = 15
    A = ora.stencil_q1_rotated(n, 5 * math.pi / 12, 0.01)
    assert np.ptp(A[4]) < 1e-14 * A[4].max()  # the Q1 diagonal does not depend on the node
    M = ora.stencil_to_dense(A)
    lam, V = np.linalg.eigh(M)
    W = np.zeros((25, n, n))
    W[12] = 2.0 / 3.0
    for q in range(0, n * n, 7):
        v = V[:, q].reshape(n, n)
        g = v - ora.apply_smoother5(A, W, ora.matvec(A, v))
        assert np.linalg.norm(g) == pytest.approx(abs(1 - (2.0 / 3.0) * lam[q] / A[4, 0, 0]), rel=1e-10, abs=1e-13)
