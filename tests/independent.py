"""Independent constructions used to pin the oracle (test code only).

Nothing here calls the oracle: these build the same mathematical objects by
a different route (global finite-element assembly by Gauss quadrature,
Kronecker-product transfer matrices, a sparse-matrix V-cycle), so that a
mistake in the oracle's stencil-form code shows up as a mismatch.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def fe_q1_matrix(n: int, k11, k12, k22) -> sp.csr_matrix:
    """Global Q1 stiffness on the n x n interior nodes of the unit square,
    assembled element by element with 2x2 Gauss quadrature.  Cell (I, J),
    I, J = 0..n, spans nodes (I-1..I, J-1..J); k** are [(n+1), (n+1)] per
    cell.  The 2-D stiffness does not depend on h, so every element is
    integrated on the unit reference square."""
    g = np.array([-1.0, 1.0]) / np.sqrt(3.0) * 0.5 + 0.5  # Gauss points on [0, 1]
    # reference bilinear basis on [0,1]^2: local node (a, b), a, b in {0, 1}
    def grad(a, b, x, y):
        fx = (1 - x) if a == 0 else x
        fy = (1 - y) if b == 0 else y
        dfx = -1.0 if a == 0 else 1.0
        dfy = -1.0 if b == 0 else 1.0
        return np.array([dfx * fy, fx * dfy])
    local = [(0, 0), (1, 0), (0, 1), (1, 1)]
    rows, cols, vals = [], [], []
    for J in range(n + 1):
        for I in range(n + 1):
            K = np.array([[k11[J, I], k12[J, I]], [k12[J, I], k22[J, I]]])
            Ke = np.zeros((4, 4))
            for x in g:
                for y in g:
                    G = [grad(a, b, x, y) for (a, b) in local]
                    for p in range(4):
                        for q in range(4):
                            Ke[p, q] += 0.25 * G[p] @ K @ G[q]
            nodes = [(I - 1 + a, J - 1 + b) for (a, b) in local]
            for p, (ip, jp) in enumerate(nodes):
                if not (0 <= ip < n and 0 <= jp < n):
                    continue
                for q, (iq, jq) in enumerate(nodes):
                    if not (0 <= iq < n and 0 <= jq < n):
                        continue
                    rows.append(jp * n + ip)
                    cols.append(jq * n + iq)
                    vals.append(Ke[p, q])
    return sp.csr_matrix((vals, (rows, cols)), shape=(n * n, n * n))


def stencil_field_to_csr(A: np.ndarray) -> sp.csr_matrix:
    """Sparse matrix of a [9, n, n] stencil field (row p = j*n + i)."""
    n = A.shape[1]
    rows, cols, vals = [], [], []
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            c = 3 * (dy + 1) + (dx + 1)
            for j in range(n):
                for i in range(n):
                    ii, jj = i + dx, j + dy
                    if 0 <= ii < n and 0 <= jj < n:
                        rows.append(j * n + i)
                        cols.append(jj * n + ii)
                        vals.append(A[c, j, i])
    return sp.csr_matrix((vals, (rows, cols)), shape=(n * n, n * n))


def prolongation_1d(nc: int) -> np.ndarray:
    """Linear interpolation from nc coarse to 2nc+1 fine interior nodes."""
    n = 2 * nc + 1
    P = np.zeros((n, nc))
    for I in range(nc):
        P[2 * I, I] = 0.5
        P[2 * I + 1, I] = 1.0
        P[2 * I + 2, I] = 0.5
    return P


def prolongation_2d(nc: int) -> sp.csr_matrix:
    p = sp.csr_matrix(prolongation_1d(nc))
    return sp.kron(p, p).tocsr()   # index j*n + i: kron(y, x)


def restriction_2d(nc: int) -> sp.csr_matrix:
    return (prolongation_2d(nc).T / 4.0).tocsr()


class SparseVCycle:
    """Assembled-matrix V-cycle: Galerkin levels by sparse products,
    damped Jacobi, dense solve on the coarsest level (numpy.linalg.solve)."""

    def __init__(self, A0: sp.csr_matrix, n: int, coarsest: int = 7):
        self.A = [A0.tocsr()]
        self.P = []
        m = n
        while m > coarsest:
            mc = (m - 1) // 2
            P = prolongation_2d(mc)
            R = restriction_2d(mc)
            self.P.append((P, R))
            self.A.append((R @ self.A[-1] @ P).tocsr())
            m = mc
        self.Ac = self.A[-1].toarray()

    def vcycle(self, l, r, nu1, nu2, omega):
        if l == len(self.A) - 1:
            return np.linalg.solve(self.Ac, r)
        A = self.A[l]
        d = A.diagonal()
        e = np.zeros_like(r)
        for _ in range(nu1):
            e = e + omega * (r - A @ e) / d
        P, R = self.P[l]
        ec = self.vcycle(l + 1, R @ (r - A @ e), nu1, nu2, omega)
        e = e + P @ ec
        for _ in range(nu2):
            e = e + omega * (r - A @ e) / d
        return e

    def solve(self, f, tol, maxit, nu1, nu2, omega=2.0 / 3.0):
        A = self.A[0]
        u = np.zeros_like(f)
        fn = np.linalg.norm(f)
        hist = []
        for k in range(maxit + 1):
            r = f - A @ u
            hist.append(np.linalg.norm(r) / fn)
            if hist[-1] <= tol or k == maxit:
                break
            u = u + self.vcycle(0, r, nu1, nu2, omega)
        return u, np.array(hist)
