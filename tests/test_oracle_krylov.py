"""Pins of the oracle's flexible GMRES (oracle/krylov.py) against what the
definition of GMRES fixes independently of its Arnoldi implementation."""
import numpy as np
import pytest

import mg_inputs
import oracle as ora
from oracle.krylov import fgmres


def _rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300)


def _problem(n, theta=0.7, eps=0.05, seed=3):
    A = ora.stencil_q1_rotated(n, theta, eps)
    f = mg_inputs.rhs_uniform(n, seed)
    return A, f


def test_matches_explicit_krylov_minimisation():
    # Right-preconditioned GMRES after m steps from u0 = 0: u_m = M K c with K a
    # basis of span{f, (AM) f, ..., (AM)^{m-1} f} and c minimising ||f - A M K c||.
    # The basis is built here from the explicit power sequence (QR, no Arnoldi).
    n = 15
    A, f = _problem(n)
    h = ora.Hierarchy(A)
    M = lambda r: h.vcycle(r, 1, 1)  # a linear operator (damped Jacobi smoother)
    AM = lambda x: ora.matvec(A, M(x))
    for m in (1, 2, 3, 5):
        cols = [f.ravel() / np.linalg.norm(f)]
        for _ in range(m - 1):
            v = AM(cols[-1].reshape(n, n)).ravel()
            cols.append(v / np.linalg.norm(v))
        K, _ = np.linalg.qr(np.array(cols).T)
        MK = np.array([M(K[:, q].reshape(n, n)).ravel() for q in range(m)]).T
        AMK = np.array([ora.matvec(A, MK[:, q].reshape(n, n)).ravel() for q in range(m)]).T
        c = np.linalg.lstsq(AMK, f.ravel(), rcond=None)[0]
        u_ref = (MK @ c).reshape(n, n)
        u, k, hist, _ = fgmres(lambda x: ora.matvec(A, x), M, f, 0.0, m, restart=m)
        assert k == m
        assert _rel(u, u_ref) <= 1e-8
        r_ref = np.linalg.norm(f.ravel() - AMK @ c) / np.linalg.norm(f)
        assert hist[-1] == pytest.approx(r_ref, rel=1e-8)


def test_exact_in_n_steps_without_preconditioner():
    # N = 9 unknowns: the Krylov space of dimension 9 is the whole space
    n = 3
    A, f = _problem(n, 0.3, 0.5, 1)
    u, k, hist, conv = fgmres(lambda x: ora.matvec(A, x), lambda r: r, f, 1e-12, 9, restart=9)
    dense = ora.stencil_to_dense(A)
    assert conv and k <= 9
    assert _rel(u.ravel(), np.linalg.solve(dense, f.ravel())) <= 1e-10


def test_residuals_monotone_within_a_cycle_and_restarts_continue():
    n = 31
    A, f = _problem(n, 1.1, 0.01, 2)
    h = ora.Hierarchy(A)
    u, k, hist, conv = fgmres(lambda x: ora.matvec(A, x), lambda r: h.vcycle(r, 1, 1), f, 1e-10, 200, restart=5)
    assert conv
    for c0 in range(0, k, 5):  # within each cycle of 5 the minimised residual cannot grow
        seg = hist[c0:c0 + 6]
        assert np.all(np.diff(seg) <= 1e-12)
    true = np.linalg.norm(f - ora.matvec(A, u)) / np.linalg.norm(f)
    assert true <= 1e-10
    assert hist[-1] == pytest.approx(true, rel=1e-3, abs=1e-13)


def test_never_worse_than_the_stationary_iteration():
    # With a linear preconditioner M, the k-th stationary iterate
    # u_k = M sum_{i<k} (I - A M)^i f lies in the space GMRES minimises over,
    # so (without restarts) GMRES's residual is never larger.
    n = 63
    A, f = _problem(n, np.pi / 6, 0.01, 0)
    h = ora.Hierarchy(A)
    _, ks, hist_s, _ = h.solve(f, 0.0, 25, 1, 1)
    _, kg, hist_g, _ = fgmres(lambda x: ora.matvec(A, x), lambda r: h.vcycle(r, 1, 1), f, 0.0, 25, restart=25)
    assert ks == kg == 25
    assert np.all(hist_g[:26] <= hist_s[:26] * (1 + 1e-10))
    assert hist_g[25] < 0.1 * hist_s[25]  # and on this problem far smaller


def test_zero_rhs_and_exact_start():
    n = 7
    A, f = _problem(n)
    u, k, hist, conv = fgmres(lambda x: ora.matvec(A, x), lambda r: r, np.zeros_like(f), 1e-8, 10)
    assert conv and k == 0 and not u.any()
    exact = np.linalg.solve(ora.stencil_to_dense(A), f.ravel()).reshape(n, n)
    u, k, hist, conv = fgmres(lambda x: ora.matvec(A, x), lambda r: r, f, 1e-8, 10, u0=exact)
    assert conv and k == 0
