"""Pins of the oracle's discretisations against independent constructions."""
import math
import os

import numpy as np
import pytest

import mg_inputs
from tests.independent import fe_q1_matrix, stencil_field_to_csr

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _interior(n):
    return (slice(None), slice(1, n - 1), slice(1, n - 1))


def test_q1_identity_tensor_closed_form(ora):
    # K = I: (1/3)[-1 -1 -1; -1 8 -1; -1 -1 -1] in the interior
    n = 15
    A = ora.stencil_q1_rotated(n, 0.3, 1.0)
    expect = np.array([-1, -1, -1, -1, 8, -1, -1, -1, -1]) / 3.0
    got = A[:, 7, 7]
    assert np.allclose(got, expect, atol=1e-15)


def test_q1_matches_paper_isotropic_formula(ora):
    # section 4: cellwise isotropic g gives the printed nine-point stencil
    table = {}
    with open(os.path.join(GOLDEN, "paper_q1_isotropic_stencil.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            name, *vals = line.split()
            table[name] = np.array([float(v) for v in vals])
    n = 9
    rng = np.random.default_rng(3)
    g = rng.uniform(0.5, 2.0, (n + 1, n + 1))
    A = ora.stencil_q1_cells(n, g, np.zeros_like(g), g)
    # the paper's u_rc: r = 1 (bottom, j-1) .. 3 (top, j+1)?  Its figure is
    # missing; the formula is symmetric under the choice, so take row index
    # r <-> dy = r-2 and column c <-> dx = c-2; g1 at corner u11 is then the
    # SW cell, g2 (u13) the SE cell, g3 (u31) the NW cell, g4 (u33) the NE cell.
    for j in range(n):
        for i in range(n):
            gs = np.array([g[j, i], g[j, i + 1], g[j + 1, i], g[j + 1, i + 1]])
            for r in range(1, 4):
                for c in range(1, 4):
                    dy, dx = r - 2, c - 2
                    ch = 3 * (dy + 1) + (dx + 1)
                    inside = 0 <= i + dx < n and 0 <= j + dy < n
                    expect = table[f"u{r}{c}"] @ gs if inside else 0.0
                    assert A[ch, j, i] == pytest.approx(expect, abs=1e-14)


@pytest.mark.parametrize("n", [7, 15])
def test_q1_tensor_matches_gauss_quadrature_assembly(ora, n):
    rng = np.random.default_rng(n)
    th = rng.uniform(0, math.pi, (n + 1, n + 1))
    ep = 10.0 ** rng.uniform(-3, 0, (n + 1, n + 1))
    c, s = np.cos(th), np.sin(th)
    k11, k12, k22 = c * c + ep * s * s, c * s * (1 - ep), s * s + ep * c * c
    A = ora.stencil_q1_cells(n, k11, k12, k22)
    M_fe = fe_q1_matrix(n, k11, k12, k22).toarray()
    M_st = stencil_field_to_csr(A).toarray()
    assert np.abs(M_fe - M_st).max() <= 1e-14 * np.abs(M_fe).max()


def test_q1_rotated_is_constant_tensor(ora):
    n, theta, eps = 15, 0.7, 0.02
    A = ora.stencil_q1_rotated(n, theta, eps)
    c, s = math.cos(theta), math.sin(theta)
    one = np.ones((n + 1, n + 1))
    B = ora.stencil_q1_cells(n, (c * c + eps * s * s) * one, c * s * (1 - eps) * one, (s * s + eps * c * c) * one)
    assert np.array_equal(A, B)


def test_q1_rotated_worked_values_c1(ora):
    # closed form for theta = pi/6, eps = 0.01 (k11 = 0.7525, k12 = 0.428683..., k22 = 0.2575)
    A = ora.stencil_q1_rotated(63, math.pi / 6, 0.01)
    c, s, eps = math.cos(math.pi / 6), math.sin(math.pi / 6), 0.01
    k11, k12, k22 = c * c + eps * s * s, c * s * (1 - eps), s * s + eps * c * c
    got = A[:, 30, 30]
    assert got[4] == pytest.approx(4 * (k11 + k22) / 3, abs=1e-15)
    assert got[4] == pytest.approx(1.346667, abs=1e-6)
    assert got[7] == pytest.approx(0.079167, abs=1e-6) and got[1] == pytest.approx(got[7], abs=1e-15)
    assert got[5] == pytest.approx(-0.415833, abs=1e-6) and got[3] == pytest.approx(got[5], abs=1e-15)
    assert got[8] == pytest.approx(-0.382675, abs=1e-6) and got[0] == pytest.approx(got[8], abs=1e-15)
    assert got[6] == pytest.approx(0.046008, abs=1e-6) and got[2] == pytest.approx(got[6], abs=1e-15)
    assert abs(got.sum()) < 1e-14


def test_q1_consistency_on_quadratics(ora):
    # sum_q A_pq x_q^2 = -2 k11 h^2 and sum_q A_pq x_q y_q = -2 k12 h^2 at interior nodes
    # (the stiffness row applied to a quadratic equals the integral of -div(K grad u) phi_p)
    n, theta, eps = 31, 1.1, 0.05
    A = ora.stencil_q1_rotated(n, theta, eps)
    h = 1.0 / (n + 1)
    x = (np.arange(n) + 1) * h
    X, Y = np.meshgrid(x, x)
    c, s = math.cos(theta), math.sin(theta)
    k11, k12 = c * c + eps * s * s, c * s * (1 - eps)
    y1 = ora.matvec(A, X * X)
    y2 = ora.matvec(A, X * Y)
    assert np.allclose(y1[1:-1, 1:-1], -2 * k11 * h * h, atol=1e-14)
    assert np.allclose(y2[1:-1, 1:-1], -2 * k12 * h * h, atol=1e-14)


def test_q1_mirror_symmetry(ora):
    n = 15
    A = ora.stencil_q1_rotated(n, 0.4, 0.1)
    B = ora.stencil_q1_rotated(n, math.pi - 0.4, 0.1)
    # mirror x -> -x: channel (dy, dx) -> (dy, -dx), node i -> n-1-i
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            ca, cb = 3 * (dy + 1) + (dx + 1), 3 * (dy + 1) + (-dx + 1)
            assert np.allclose(A[ca], B[cb][:, ::-1], atol=1e-15)


def test_q1_boundary_entries_zero_and_symmetric(ora):
    n = 15
    A = ora.stencil_q1_rotated(n, 2.0, 0.003)
    M = stencil_field_to_csr(A).toarray()
    assert np.abs(M - M.T).max() < 1e-15
    assert np.all(A[0:3, 0, :] == 0) and np.all(A[6:9, n - 1, :] == 0)
    assert np.all(A[[0, 3, 6], :, 0] == 0) and np.all(A[[2, 5, 8], :, n - 1] == 0)
    assert np.all(np.linalg.eigvalsh(M) > 0)


def test_cellavg5_constant_is_5pt_laplacian(ora):
    n = 15
    A = ora.stencil_cellavg5(n, 2.5 * np.ones((n + 1, n + 1)))
    assert np.allclose(A[:, 7, 7], 2.5 * np.array([0, -1, 0, -1, 4, -1, 0, -1, 0]), atol=1e-15)


def test_cellavg5_matches_edge_energy_assembly(ora):
    # A = Hessian of (1/2) sum_edges a_e (u_p - u_q)^2, a_e = mean of the two cells on the edge
    n = 9
    rng = np.random.default_rng(1)
    a = np.exp(rng.standard_normal((n + 1, n + 1)))
    A = ora.stencil_cellavg5(n, a)
    N = n * n
    M = np.zeros((N, N))

    def node(i, j):
        return j * n + i if (0 <= i < n and 0 <= j < n) else None

    # horizontal edges (i,j)-(i+1,j), i = -1..n-1: cells below (i+1, j) and above (i+1, j+1)
    for j in range(n):
        for i in range(-1, n):
            ae = 0.5 * (a[j, i + 1] + a[j + 1, i + 1])
            p, q = node(i, j), node(i + 1, j)
            for u, v in ((p, q), (q, p)):
                if u is not None:
                    M[u, u] += ae
                    if v is not None:
                        M[u, v] -= ae
    # vertical edges (i,j)-(i,j+1): cells left (i, j+1) and right (i+1, j+1)
    for i in range(n):
        for j in range(-1, n):
            ae = 0.5 * (a[j + 1, i] + a[j + 1, i + 1])
            p, q = node(i, j), node(i, j + 1)
            for u, v in ((p, q), (q, p)):
                if u is not None:
                    M[u, u] += ae
                    if v is not None:
                        M[u, v] -= ae
    assert np.abs(stencil_field_to_csr(A).toarray() - M).max() < 1e-13


@pytest.mark.parametrize("kind", ["lshape", "cylinder"])
def test_masked_stencil_is_the_interior_block(ora, kind):
    # the operator of the domain = the principal submatrix of the square's operator on the
    # inside nodes; the outside nodes decouple with their own centre entry
    n = 15
    A = ora.stencil_q1_rotated(n, math.pi / 4, 0.01)
    mask = mg_inputs.domain_mask(n, kind).ravel().astype(bool)
    M = ora.stencil_to_dense(ora.stencil_mask(A, mask.reshape(n, n)))
    F = ora.stencil_to_dense(A)
    inn, out = np.flatnonzero(mask), np.flatnonzero(~mask)
    assert 0 < len(out) < n * n
    assert np.array_equal(M[np.ix_(inn, inn)], F[np.ix_(inn, inn)])
    assert not M[np.ix_(inn, out)].any() and not M[np.ix_(out, inn)].any()
    assert np.array_equal(M[np.ix_(out, out)], np.diag(np.diag(F)[out]))
    # the domain's solution: zero outside, the interior block's solve inside
    f = mg_inputs.rhs_uniform(n, 0).ravel() * mask
    u = np.linalg.solve(M, f)
    assert not u[out].any()
    assert np.allclose(u[inn], np.linalg.solve(F[np.ix_(inn, inn)], f[inn]), rtol=1e-12, atol=1e-14)


def test_domain_masks():
    n = 63
    sq, ls, cy = (mg_inputs.domain_mask(n, k) for k in ("square", "lshape", "cylinder"))
    assert sq.all()
    # the removed quadrant: nodes with x, y >= 1/2 (index >= 31 on h = 1/64)
    assert ls.sum() == n * n - 32 * 32 and not ls[31:, 31:].any() and ls[:31, :].all()
    # the disk of radius 1/5 about the centre: about pi r^2 / h^2 nodes
    removed = n * n - cy.sum()
    assert abs(removed - math.pi * 0.04 * 64 ** 2) < 0.05 * math.pi * 0.04 * 64 ** 2
    assert cy[0, :].all() and cy[:, 0].all() and not cy[31, 31]
