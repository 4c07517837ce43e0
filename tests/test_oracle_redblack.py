"""Pins of the red-black coarsening oracle (oracle/redblack.py, section 6.1):
the paper's printed transfer stencils, R = P^T/2, linear interpolation, a
hand-worked Galerkin level of the five-point Laplacian, the A-orthogonal
projection of the coarse correction, SPD levels, the smoother against torch,
the cycle against the dense two-level operator, the solution against a
sparse direct solve, the observed rate against the spectral radius, and the
Algorithm 2 recursion and gradient against the cycle and central differences."""
import math
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import mg_inputs
import oracle as ora
from oracle import redblack as rb

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        key, *vals = line.split()
        rows.setdefault(key, []).append([float(v) for v in vals])
    return rows


def _q1(n, theta=math.pi / 3, eps=1e-2):
    return ora.stencil_q1_rotated(n, theta, eps)


def _lap5(n):
    A = np.zeros((9, n, n))
    A[4] = 4.0
    for c in (1, 3, 5, 7):
        A[c] = -1.0
    A[1][0, :] = 0.0
    A[7][n - 1, :] = 0.0
    A[3][:, 0] = 0.0
    A[5][:, n - 1] = 0.0
    return A


# ------------------------------------------------------------------ transfers
@pytest.mark.parametrize("kind", [rb.FULL, rb.CHECKER])
def test_transfer_stencils_are_the_papers(kind):
    g = _golden("paper_redblack_transfer_stencils.txt")
    Rs = np.array(g["restriction"]) * g["restriction_scale"][0][0]
    Ps = np.array(g["prolongation"]) * g["prolongation_scale"][0][0]
    N = 15
    R, P = rb.restriction(N, kind), rb.prolongation(N, kind)
    if kind == rb.FULL:  # coarse point (6, 8) of the same array; mesh axes = grid axes
        fi, fj, q = 6, 8, 8 * N + 6
        axes = {(0, 0): (1, 1), (1, 0): (1, 2), (-1, 0): (1, 0), (0, 1): (2, 1), (0, -1): (0, 1)}
    else:  # coarse node (3, 2) of the 7 x 7 grid on fine node (7, 5); mesh axes = diagonals
        Nc = (N - 1) // 2
        fi, fj, q = 7, 5, 2 * Nc + 3
        axes = {(0, 0): (1, 1), (1, 1): (1, 2), (-1, -1): (1, 0), (-1, 1): (2, 1), (1, -1): (0, 1)}
    row = R.getrow(q).toarray().reshape(N, N)
    col = P.getcol(q).toarray().reshape(N, N)
    assert np.count_nonzero(row) == 5 and np.count_nonzero(col) == 5
    for (dx, dy), (ky, kx) in axes.items():
        assert row[fj + dy, fi + dx] == Rs[ky, kx]
        assert col[fj + dy, fi + dx] == Ps[ky, kx]


@pytest.mark.parametrize("N,kind", [(15, rb.FULL), (15, rb.CHECKER), (7, rb.CHECKER), (3, rb.FULL)])
def test_restriction_is_half_the_transposed_prolongation(N, kind):
    R, P = rb.restriction(N, kind), rb.prolongation(N, kind)
    assert abs(R - P.T / 2).max() == 0.0


@pytest.mark.parametrize("kind", [rb.FULL, rb.CHECKER])
def test_interpolation_reproduces_linear_functions(kind):
    N = 31
    P = rb.prolongation(N, kind)
    pts, Nc, _ = rb._coarse_points(N, kind)
    lin = lambda i, j: 0.3 + 1.7 * i - 0.6 * j
    xc = np.zeros(Nc * Nc)
    for fi, fj, q in pts:
        xc[q] = lin(fi, fj)
    y = (P @ xc).reshape(N, N)
    mask = rb.point_mask(N, kind)
    j, i = np.mgrid[0:N, 0:N]
    inner = mask & (i >= 2) & (i < N - 2) & (j >= 2) & (j < N - 2)
    assert inner.sum() > 100
    assert np.abs(y[inner] - lin(i, j)[inner]).max() <= 1e-12
    assert np.all(y[~mask] == 0.0)


# ------------------------------------------------------------------- Galerkin
def test_galerkin_level_of_the_five_point_laplacian_is_the_worked_stencil():
    g = _golden("redblack_galerkin_5pt.txt")
    scale = g["scale"][0][0]
    expect = {(int(dx), int(dy)): v * scale for dx, dy, v in g["offset"]}
    n = 31
    h = rb.RBHierarchy(_lap5(n), 2)
    A1 = h.A[1]
    for fi, fj in [(15, 15), (10, 12), (20, 8)]:
        row = A1.getrow(fj * n + fi).tocoo()
        got = {(int(c % n) - fi, int(c // n) - fj): v for c, v in zip(row.col, row.data) if v != 0.0}
        assert set(got) == set(expect)
        for d, v in expect.items():
            assert got[d] == pytest.approx(v, abs=1e-15)


def _active(h, level):
    return np.flatnonzero(h.masks[level].reshape(-1))


@pytest.mark.parametrize("level", [0, 1, 2])
def test_coarse_correction_is_an_A_orthogonal_projection(level):
    h = rb.RBHierarchy(_q1(15, 1.0, 0.05), 4)
    ia, ic = _active(h, level), _active(h, level + 1)
    A = h.A[level].toarray()[np.ix_(ia, ia)]
    Ac = h.A[level + 1].toarray()[np.ix_(ic, ic)]
    P = h.P[level].toarray()[np.ix_(ia, ic)]
    R = h.R[level].toarray()[np.ix_(ic, ia)]
    assert np.allclose(Ac, R @ A @ P, atol=1e-14)
    C = P @ np.linalg.solve(Ac, R @ A)
    assert np.abs(C @ C - C).max() <= 1e-12
    AC = A @ C
    assert np.abs(AC - AC.T).max() <= 1e-12


def test_every_level_is_symmetric_positive_definite():
    h = rb.RBHierarchy(_q1(31, math.pi / 3, 1e-3), 7)
    assert [s for s in h.shapes] == [(31, "full"), (31, "checker"), (15, "full"), (15, "checker"),
                                     (7, "full"), (7, "checker"), (3, "full")]
    for l in range(h.num_levels):
        ia = _active(h, l)
        M = h.A[l].toarray()
        assert np.abs(M - M.T).max() <= 1e-13 * np.abs(M).max()
        inactive = np.setdiff1d(np.arange(M.shape[0]), ia)
        assert np.all(M[inactive] == 0.0) and np.all(M[:, inactive] == 0.0)
        assert np.linalg.eigvalsh(M[np.ix_(ia, ia)]).min() > 0.0


# ------------------------------------------------------------------ smoothers
def test_two_layer_smoother_matches_torch_conv2d():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    phi = rng.normal(size=(2, 3, 3))
    for kind in (rb.FULL, rb.CHECKER):
        N = 15
        mask = rb.point_mask(N, kind)
        x = rng.normal(size=(N, N)) * mask
        t = torch.tensor((x * mask)[None, None])
        k1 = torch.tensor(phi[0][None, None])
        k2 = torch.tensor(phi[1][None, None])
        y = torch.nn.functional.conv2d(torch.nn.functional.conv2d(t, k1, padding=1), k2, padding=1)[0, 0].numpy()
        assert np.abs(rb.smoother_apply(phi, x, mask) - y * mask).max() <= 1e-14


def test_jacobi_stack_is_damped_jacobi_on_the_finest_level():
    n = 31
    A = _q1(n)
    h = rb.RBHierarchy(A, 5)
    r = mg_inputs.rhs_uniform(n, 2)
    e_j = h.vcycle(r)
    h.set_smoother(0, rb.jacobi_stack(A[4, 0, 0]))
    assert np.abs(h.vcycle(r) - e_j).max() <= 1e-14 * np.abs(e_j).max()


# -------------------------------------------------------------------- V-cycle
@pytest.mark.parametrize("nlevels", [2, 3])
def test_cycle_equals_the_dense_two_level_operator(nlevels):
    # two levels: full 15 -> checkerboard 15 (solved directly); three: the checkerboard's own
    # coarse correction is a cycle, so the dense operator recurses once more
    n = 15
    h = rb.RBHierarchy(_q1(n, 0.4, 0.02), nlevels)
    rng = np.random.default_rng(7)
    h.set_smoother(0, rb.jacobi_stack(_q1(n, 0.4, 0.02)[4, 0, 0]) + 0.01 * rng.normal(size=(2, 3, 3)))

    def dense_cycle(level):
        ia = _active(h, level)
        A = h.A[level].toarray()[np.ix_(ia, ia)]
        if level == h.num_levels - 1:
            return np.linalg.inv(A)  # e = A^-1 r
        m = ia.size
        N = h.level_n(level)
        H = np.zeros((m, m))
        for c, p in enumerate(ia):
            x = np.zeros(N * N)
            x[p] = 1.0
            H[:, c] = h.apply_smoother(level, x.reshape(N, N)).reshape(-1)[ia]
        ic = _active(h, level + 1)
        P = h.P[level].toarray()[np.ix_(ia, ic)]
        R = h.R[level].toarray()[np.ix_(ic, ia)]
        Bc = dense_cycle(level + 1)
        S = np.eye(m) - H @ A
        # e = V r: pre-smooth, coarse correction with the coarse cycle, post-smooth
        E = S @ (np.eye(m) - P @ Bc @ R @ A) @ S  # error propagation
        return (np.eye(m) - E) @ np.linalg.inv(A)

    B = dense_cycle(0)
    ia = _active(h, 0)
    for c in range(0, ia.size, 17):
        r = np.zeros(n * n)
        r[ia[c]] = 1.0
        got = h.vcycle(r.reshape(n, n)).reshape(-1)[ia]
        assert np.abs(got - B[:, c]).max() <= 1e-12 * np.abs(B[:, c]).max()


def test_solve_reaches_the_direct_solution():
    n = 31
    A = _q1(n, math.pi / 3, 1e-2)
    h = rb.RBHierarchy(A, 7)
    f = mg_inputs.rhs_uniform(n, 0)
    u, k, hist, conv = h.solve(f, 1e-11, 3000)
    assert conv and 5 < k < 3000
    exact = spla.spsolve(rb.operator_matrix(A).tocsc(), f.reshape(-1)).reshape(n, n)
    assert np.abs(u - exact).max() <= 1e-9 * np.abs(exact).max()


def test_observed_rate_is_the_spectral_radius():
    n = 15
    A = _q1(n, 0.7, 0.05)
    h = rb.RBHierarchy(A, 5)
    N2 = n * n
    E = np.zeros((N2, N2))
    for c in range(N2):
        x = np.zeros(N2)
        x[c] = 1.0
        E[:, c] = x - h.vcycle(h.matvec(0, x.reshape(n, n))).reshape(-1)
    rho = np.abs(np.linalg.eigvals(E)).max()
    assert 0.05 < rho < 0.99
    f = mg_inputs.rhs_uniform(n, 1)
    _, k, hist, conv = h.solve(f, 1e-300, 40)
    tail = hist[25:41]  # well before round-off (rho^40 ~ 1e-8)
    rate = (tail[-1] / tail[0]) ** (1.0 / (len(tail) - 1))
    assert rate == pytest.approx(rho, rel=2e-3)


# ---------------------------------------------------------------- Algorithm 2
@pytest.mark.parametrize("level", [0, 1])
def test_alpha_forward_is_the_cycle_iteration(level):
    n = 15
    h = rb.RBHierarchy(_q1(n, 1.1, 0.03), 5)
    N = h.level_n(level)
    mask = h.masks[level]
    rng = np.random.default_rng(level)
    phi = rb.jacobi_stack(h.diag(level)[N // 2, N // 2]) + 0.02 * rng.normal(size=(2, 3, 3))
    f = rng.uniform(-1, 1, (N, N)) * mask
    u0 = rng.normal(size=(N, N)) * mask
    u = h.alpha_forward(level, phi, f, u0, 3)
    h.set_smoother(level, phi)
    ref = u0.copy()
    for _ in range(3):
        ref = ref + h.vcycle(f - h.matvec(level, ref), level)
    assert np.abs(u - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("level", [0, 1, 2])
def test_alpha_gradient_matches_central_differences(level):
    n = 15
    h = rb.RBHierarchy(_q1(n, 0.5, 0.05), 5)
    N = h.level_n(level)
    mask = h.masks[level]
    rng = np.random.default_rng(10 + level)
    phi = rb.jacobi_stack(h.diag(level)[N // 2, N // 2]) + 0.05 * rng.normal(size=(2, 3, 3))
    f = rng.uniform(-1, 1, (N, N)) * mask
    u0 = rng.normal(size=(N, N)) * mask
    u_star = rng.normal(size=(N, N)) * mask
    L, g = h.alpha_loss_and_grad(level, phi, f, u0, u_star, 2)
    assert L == pytest.approx(np.linalg.norm(h.alpha_forward(level, phi, f, u0, 2) - u_star), rel=1e-14)
    w = phi.reshape(-1)
    for j in range(rb.NWEIGHTS):
        d = 1e-6
        wp, wm = w.copy(), w.copy()
        wp[j] += d
        wm[j] -= d
        Lp = np.linalg.norm(h.alpha_forward(level, wp, f, u0, 2) - u_star)
        Lm = np.linalg.norm(h.alpha_forward(level, wm, f, u0, 2) - u_star)
        fd = (Lp - Lm) / (2 * d)
        assert abs(fd - g[j]) <= 1e-6 * max(1.0, np.abs(g).max()), (j, fd, g[j])
